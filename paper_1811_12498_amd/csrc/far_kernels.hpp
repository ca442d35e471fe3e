// Far-field kernel: one wavefront per group of 64 Morton-consecutive targets walks the
// group's far list of (cluster, lane mask) entries; lanes whose target accepted the
// cluster (eq. MAC) evaluate eq. S_final + eq. T_final through the scaled recurrence
// and the G/E contraction of stk_math.hpp.  The cluster index is wave-uniform, so its
// block is read through the scalar cache and broadcast to the lanes as SGPR operands.
// Workgroups are numbered so that each XCD (8 per chip, each with its own L2) runs a
// contiguous range of groups, which share most of their clusters.
#pragma once

#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {

struct FarArgs {
    const double *tpos;      // (m,3) sorted targets
    int64_t m;
    const int32_t *off;      // (ngroups + 1)
    const int32_t *node;     // entries
    const uint64_t *mask;
    const double *center;    // (nn,3)
    const double *rho;       // (nn)
    const void *wblk;        // (nn, 6 nG) in T: each cluster's G/E stream
    const double *unear;     // (m,3) sorted near-field velocity
    const int32_t *tperm;    // sorted -> caller index
    double *u_out;           // (m,3) caller order
    int32_t ngroups;
};

// block index -> group: XCD x = blockIdx % 8 gets groups [x * per, (x + 1) * per)
__device__ inline int32_t xcd_group(int32_t ngroups) {
    const int32_t per = (ngroups + 7) >> 3;
    return int32_t(blockIdx.x & 7) * per + int32_t(blockIdx.x >> 3);
}
inline unsigned xcd_blocks(int32_t ngroups) { return unsigned(((ngroups + 7) >> 3) << 3); }

template <int P, typename T>
__global__ __launch_bounds__(64) void k_far(FarArgs a) {
    constexpr int NG = nidx(P + 1);
    const int32_t g = xcd_group(a.ngroups);
    if (g >= a.ngroups) return;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    const bool valid = t < a.m;
    double x0 = 0, x1 = 0, x2 = 0;
    if (valid) {
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    Comp<T> acc[3];
    const T *__restrict__ wb = static_cast<const T *>(a.wblk);
    const int32_t e0 = a.off[g], e1 = a.off[g + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t c = __builtin_amdgcn_readfirstlane(a.node[e]);
        const uint64_t mk = a.mask[e];
        if ((mk >> lane) & 1ull) {
            const double d0 = x0 - a.center[3 * c], d1 = x1 - a.center[3 * c + 1], d2 = x2 - a.center[3 * c + 2];
            const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
            const double rinv = 1.0 / sqrt(R2);
            const T dh[3] = {T(d0 * rinv), T(d1 * rinv), T(d2 * rinv)};
            const T tt = T(a.rho[c] * rinv);
            T accG[3], accF[3];
            FarEval<P, T>::run(dh, tt, wb + size_t(c) * 6 * NG, accG, accF);
            T u[3];
            far_velocity(accG, accF, T(rinv), u);
            acc[0].add(u[0]);
            acc[1].add(u[1]);
            acc[2].add(u[2]);
        }
    }
    if (valid) {
        const int64_t o = a.tperm[t];
        a.u_out[3 * o] = acc[0].value() + a.unear[3 * t];
        a.u_out[3 * o + 1] = acc[1].value() + a.unear[3 * t + 1];
        a.u_out[3 * o + 2] = acc[2].value() + a.unear[3 * t + 2];
    }
}

template <int P, typename T> void launch_far(const FarArgs &a, hipStream_t s) {
    if (a.ngroups == 0) return;
    hipLaunchKernelGGL((k_far<P, T>), dim3(xcd_blocks(a.ngroups)), dim3(64), 0, s, a);
    STK_CHECK_LAUNCH();
}

}  // namespace stk
