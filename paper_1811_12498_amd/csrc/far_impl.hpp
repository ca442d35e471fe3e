// Far-field kernel body (instantiated per Taylor order in far_p*.hip and fark_p*.hip).
#pragma once

#include "far_kernels.hpp"

namespace stk {

// right-hand sides in blocks of KB, one block per grid row (blockIdx.y): each wave
// walks its group's far list once and shares each interaction's recurrence between the
// block's KB streams.  All resident waves work on the same block, so the streams in use
// at a time are KB per cluster (the cluster data of one block fits the XCD's L2 where
// that of all K would not).  With nsplit > 1 the list is cut into nsplit contiguous parts
// (grid z), each a wave of its own that writes its compensated sums to fpart: more, shorter
// waves, so the last round of waves on a chip with few rounds leaves less of it idle.
template <int P, typename T, int KB>
__global__ __launch_bounds__(64) void k_far(FarArgs a) {
    constexpr int WS = 6 * nidx(P + 1);
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
    // FP64 streams are read through the constant address space: the double u_out stores
    // between right-hand-side blocks would otherwise turn their uniform loads into vector
    // loads (FP32 streams cannot alias them)
    constexpr bool CAS = sizeof(T) == 8;
    using Eval = FarEval<P, T, KB, CAS>;
    const typename Eval::Ptr __restrict__ wb = (typename Eval::Ptr)(a.wblk);
    const int32_t f0 = a.off[g], f1 = a.off[g + 1];
    const int32_t h = int32_t(blockIdx.z);
    const int32_t e0 = f0 + int32_t((int64_t(f1 - f0) * h) / a.nsplit);
    const int32_t e1 = f0 + int32_t((int64_t(f1 - f0) * (h + 1)) / a.nsplit);
    const int K = a.K;
    {
        const int r0 = int(blockIdx.y) * KB;
        Comp<T> acc[KB][3];
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t c = __builtin_amdgcn_readfirstlane(a.node[e]);
            const uint64_t mk = a.mask[e];
            if (__popcll(mk) <= a.sparse_max) continue;  // done cluster major (k_far_sparse)
            if ((mk >> lane) & 1ull) {
                const double d0 = x0 - a.center[3 * c], d1 = x1 - a.center[3 * c + 1], d2 = x2 - a.center[3 * c + 2];
                const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
                const double rinv = 1.0 / sqrt(R2);
                const T dh[3] = {T(d0 * rinv), T(d1 * rinv), T(d2 * rinv)};
                const T tt = T(a.rho[c] * rinv);
                T accG[KB][3], accF[KB][3];
                Eval::run(dh, tt, wb + (size_t(c) * K + r0) * WS, accG, accF);
#pragma unroll
                for (int r = 0; r < KB; ++r) {
                    T u[3];
                    far_velocity(accG[r], accF[r], T(rinv), u);
                    acc[r][0].add(u[0]);
                    acc[r][1].add(u[1]);
                    acc[r][2].add(u[2]);
                }
            }
        }
        if (valid) {
            if (a.nsplit == 1) {
                const int64_t o = a.tperm[t];
#pragma unroll
                for (int r = 0; r < KB; ++r)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        a.u_out[(size_t(r0 + r) * a.m + o) * 3 + i] =
                            acc[r][i].value() + a.unear[(size_t(t) * K + r0 + r) * 3 + i];
            } else {
#pragma unroll
                for (int r = 0; r < KB; ++r)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        a.fpart[((size_t(h) * K + r0 + r) * a.m + t) * 3 + i] = acc[r][i].value();
            }
        }
    }
}

template <int P, typename T, int KB> void launch_far(const FarArgs &a, hipStream_t s) {
    if (a.ngroups == 0) return;
    hipLaunchKernelGGL((k_far<P, T, KB>), dim3(xcd_blocks(a.ngroups), unsigned(a.K / KB), unsigned(a.nsplit)), dim3(64),
                       0, s, a);
    STK_CHECK_LAUNCH();
}

// one wave per item: a cluster and up to 64 targets whose groups' entries for it run
// cluster major; each lane evaluates its (target, cluster) interaction for every
// right-hand side (KB of them per Taylor-coefficient recurrence) and writes the velocities
// to the interaction's slot in the target's list of cluster-major entries
template <int P, typename T, int KB> __global__ __launch_bounds__(64) void k_far_sparse(FarSparseArgs a) {
    constexpr int WS = 6 * nidx(P + 1);
    // the streams are read through the constant address space: the partial stores below
    // cannot alias them, so their uniform loads stay scalar across the loop
    using Eval = FarEval<P, T, KB, true>;
    const int32_t it = xcd_item<XCD_CHUNK_FAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int32_t c = __builtin_amdgcn_readfirstlane(a.item_node[it]);
    const int32_t i0 = a.item_i0[it];
    if (lane < a.item_i1[it] - i0) {
        const int64_t t = a.inc_tgt[i0 + lane];
        const int32_t slot = a.inc_slot[i0 + lane];
        const double d0 = a.tpos[3 * t] - a.center[3 * c], d1 = a.tpos[3 * t + 1] - a.center[3 * c + 1],
                     d2 = a.tpos[3 * t + 2] - a.center[3 * c + 2];
        const double rinv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const T dh[3] = {T(d0 * rinv), T(d1 * rinv), T(d2 * rinv)};
        const T tt = T(a.rho[c] * rinv);
        const T *wb = static_cast<const T *>(a.wblk) + size_t(c) * a.K * WS;
        T *o = static_cast<T *>(a.part) + 3 * int64_t(slot) * a.K;
        for (int r0 = 0; r0 < a.K; r0 += KB) {
            // the recurrence is redone per block of right-hand sides: opaque copies of its
            // inputs keep the compiler from hoisting all coefficients out of the loop (they
            // would not fit the register file)
            T dr[3] = {dh[0], dh[1], dh[2]}, tr = tt;
#if defined(__HIP_DEVICE_COMPILE__)
            asm("" : "+v"(dr[0]), "+v"(dr[1]), "+v"(dr[2]), "+v"(tr));
#endif
            T accG[KB][3], accF[KB][3];
            Eval::run(dr, tr, (typename Eval::Ptr)(wb + size_t(r0) * WS), accG, accF);
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                T u[3];
                far_velocity(accG[r], accF[r], T(rinv), u);
                o[3 * (r0 + r)] = u[0];
                o[3 * (r0 + r) + 1] = u[1];
                o[3 * (r0 + r) + 2] = u[2];
            }
        }
    }
}

template <int P, typename T, int KB> void launch_far_sparse(const FarSparseArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    hipLaunchKernelGGL((k_far_sparse<P, T, KB>), dim3(xcd_item_blocks<XCD_CHUNK_FAR>(a.nitems)), dim3(64), 0, s, a);
    STK_CHECK_LAUNCH();
}

}  // namespace stk
