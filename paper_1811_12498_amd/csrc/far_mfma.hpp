// Far field for K right-hand sides on the matrix cores (FP32 mixed precision).
//
// With the G/E regrouping of eq. S_final + eq. T_final (stk_math.hpp), one far
// interaction adds, for every Taylor coefficient bt^r of order <= p + 2,
//     u_i += (bt^r / R) Ghat_i^r + sum_c (r_i dh_c bt^r) Ehat_c^{r - e_i},   c = 0..2,
// i.e. four products per r whose left factors depend on the target and whose right
// factors depend on the cluster and the right-hand side.  For 16 targets and 16
// right-hand sides this is a product of a (16 targets x 4 slots) block by a
// (4 slots x 16 RHS) block per (r, i): one v_mfma_f32_16x16x4_f32 with
//     A[t][c] = r_i dh_c(t) bt^r(t)  (c < 3),   A[t][3] = bt^r(t) / R(t),
//     B[c][rr] = Ehat_c^{r - e_i}(rr) (c < 3), B[3][rr] = Ghat_i^r(rr).
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]: the four lanes of a target
// run its recurrence (Coefs, the same arithmetic as FarEval) and each multiplies by its
// own slot factor, and the cluster's B blocks are stored per (r, lane) by k_far_bm, so
// no lane exchanges data.  A wave takes one 16-target quarter of a 64-target group; the
// four quarters of a group are the four waves of a workgroup and walk the same far list,
// so a cluster's B blocks are read once into L1 for all four.  Each interaction is summed
// in a fresh accumulator and added to compensated per-lane sums.
#pragma once

#include "adjoint_far_impl.hpp"
#include "far_kernels.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {

typedef float mf32x4 __attribute__((ext_vector_type(4)));

// B blocks of one cluster and one block of 16 right-hand sides: Bm[r][lane][i], r over the
// nidx(p + 2) coefficients in graded-lex order
template <int P> __host__ __device__ constexpr int far_bm_rows() { return nidx(P + 2); }

struct FarBmArgs {
    const float *wblk;   // (nn, K, 6 nG) streams
    float *bm;           // (nn, nrb, rows, 64, 3)
    int32_t nn, K, nrb;
};

// grid (nn, nrb), 64 threads: lane l fills slot c = l / 16 for right-hand side
// rb * 16 + l % 16 (zero beyond K)
template <int P> __global__ __launch_bounds__(64) void k_far_bm(FarBmArgs a) {
    constexpr int NG = nidx(P + 1), WS = 6 * NG, ROWS = far_bm_rows<P>();
    const int32_t node = blockIdx.x;
    const int rb = blockIdx.y;
    const int lane = threadIdx.x, c = lane >> 4;
    const int rr = rb * 16 + (lane & 15);
    const bool ok = rr < a.K;
    const float *st = a.wblk + (size_t(node) * a.K + (ok ? rr : 0)) * WS;
    float *out = a.bm + ((size_t(node) * a.nrb + rb) * ROWS) * 64 * 3;
    for (int r = 0; r < ROWS; ++r) {
        int q[3];
        kof(r, q);
        const int n = q[0] + q[1] + q[2];
        for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
            if (ok) {
                if (c == 3) {
                    if (n <= P + 1) {
                        int pg, pe;
                        stream_pos(P, q, pg, pe);
                        v = st[pg + i];
                    }
                } else if (q[i] >= 1) {
                    int k[3] = {q[0], q[1], q[2]};
                    k[i] -= 1;
                    int pg, pe;
                    stream_pos(P, k, pg, pe);
                    v = st[pe + c];
                }
            }
            out[(size_t(r) * 64 + lane) * 3 + i] = v;
        }
    }
}

template <int P> struct MfmaVisit {
    const float *bm;   // this cluster's B blocks, already offset by the lane
    float fe, fg;      // slot factors: dh_c (c < 3) and 1/R (c = 3); 0 for lanes without work
    bool slot_e;       // c < 3
    mf32x4 acc[3];

    template <int Q, int N> STK_HD void coef(float bq) {
        constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = N - K1 - K2;
        constexpr int RI[3] = {K1, K2, K3};
        const float *b3 = bm + Q * 64 * 3;
        const float x = bq * (slot_e ? fe : fg);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            // slot c < 3: r_i dh_c bt^r; slot 3: bt^r / R
            const float ai = slot_e ? float(RI[i]) * x : x;
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b3[i], acc[i], 0, 0, 0);
        }
    }
    template <int N, int J> STK_HD void layer_done(const float (&)[nidx(P + 2)]) {}
    template <int N> STK_HD void order_done(const float (&)[nidx(P + 2)]) {}
};

// grid (xcd_blocks(ngroups), nrb), 256 threads: wave w = quarter w of the group
template <int P> __global__ __launch_bounds__(256) void k_far_mfma(FarArgs a, const float *__restrict__ bm, int nrb) {
    constexpr int ROWS = far_bm_rows<P>();
    const int32_t g = xcd_group(a.ngroups);
    if (g >= a.ngroups) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tl = lane & 15, c = lane >> 4;
    const int rb = blockIdx.y;
    const int64_t t = int64_t(g) * 64 + 16 * wave + tl;  // this lane's target (A row)
    const bool valid = t < a.m;
    double x0 = 0, x1 = 0, x2 = 0;
    if (valid) {
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    Comp<float> sum[3][4];
    for (int32_t e = a.off[g]; e < a.off[g + 1]; ++e) {
        const uint64_t mk = a.mask[e];
        if (((mk >> (16 * wave)) & 0xffffull) == 0) continue;  // no target of this quarter
        const int32_t cl = __builtin_amdgcn_readfirstlane(a.node[e]);
        const bool on = (mk >> (16 * wave + tl)) & 1ull;
        const double d0 = x0 - a.center[3 * cl], d1 = x1 - a.center[3 * cl + 1], d2 = x2 - a.center[3 * cl + 2];
        const double R2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double rinv = on ? 1.0 / sqrt(R2) : 0.0;
        float dh[3] = {float(d0 * rinv), float(d1 * rinv), float(d2 * rinv)};
        if (!on) dh[0] = 1.0f;  // a finite direction for lanes without work (their factors are 0)
        const float tt = on ? float(a.rho[cl] * rinv) : 0.0f;
        MfmaVisit<P> v;
        v.bm = bm + ((size_t(cl) * nrb + rb) * ROWS * 64 + lane) * 3;
        v.slot_e = c < 3;
        v.fe = on ? (c == 0 ? dh[0] : (c == 1 ? dh[1] : dh[2])) : 0.0f;
        v.fg = on ? float(rinv) : 0.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i) v.acc[i] = mf32x4{0.0f, 0.0f, 0.0f, 0.0f};
        float b[nidx(P + 2)];
        Coefs<P + 2, float, MfmaVisit<P>>::run(b, dh, tt, v);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[i][q].add(v.acc[i][q]);
    }
    // lane holds rows 4 c + q (targets 16 wave + 4 c + q of the group), column tl (RHS)
    const int r = rb * 16 + tl;
    if (r < a.K) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t tq = int64_t(g) * 64 + 16 * wave + 4 * c + q;
            if (tq < a.m) {
                const int64_t o = a.tperm[tq];
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    a.u_out[(size_t(r) * a.m + o) * 3 + i] = sum[i][q].value() + a.unear[(size_t(tq) * a.K + r) * 3 + i];
            }
        }
    }
}

template <int P> void launch_far_mfma(const FarArgs &a, DBuf &bm_buf, int32_t nn, hipStream_t s) {
    if (a.ngroups == 0) return;
    const int nrb = (a.K + 15) / 16;
    float *bm = reserve<float>(bm_buf, size_t(nn) * nrb * far_bm_rows<P>() * 64 * 3);
    FarBmArgs ba{static_cast<const float *>(a.wblk), bm, nn, a.K, nrb};
    hipLaunchKernelGGL((k_far_bm<P>), dim3(nn, nrb), dim3(64), 0, s, ba);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL((k_far_mfma<P>), dim3(xcd_blocks(a.ngroups), nrb), dim3(256), 0, s, a,
                       static_cast<const float *>(bm), nrb);
    STK_CHECK_LAUNCH();
}

}  // namespace stk
