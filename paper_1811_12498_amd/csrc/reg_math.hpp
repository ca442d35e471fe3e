// Arithmetic of the regularized particle-cluster far field, shared by the device kernel
// (regularized.hip) and compiled for the host only by the unit check of this header.
//
// With R = sqrt(|d|^2 + eps^2), d = x - y, both regularized kernels (the regularized
// Stokeslet of Cortez, Fauci and Medovikov 2005 and -1/6 of the stress of its flow,
// normalised like eqs. Stokeslet and stresslet) are x-derivatives of the one function R:
//   S^eps_ij  = delta_ij lap R - D_ij R,
//   T^eps_ijl = (1/3) D_ijl R - (1/6) (delta_ij D_l + delta_il D_j + delta_jl D_i) lap R,
// because lap R = 2/R + eps^2/R^3, D_ij R = delta_ij/R - d_i d_j/R^3 and
// D_ijl R = 3 d_i d_j d_l/R^5 - (delta_ij d_l + delta_il d_j + delta_jl d_i)/R^3.
//
// Let a^q be the Taylor coefficients of R(x - y) in y about the cluster centre
// (a^0 = R at d = x - y_c).  The coefficient at multi-index k of the x-derivative
// D^alpha R is (-1)^|alpha| ((k + alpha)! / k!) a^(k + alpha), so the order-p far field
//   u_i = sum_{||k|| <= p} [S^eps_ij]^k M_j^k + [T^eps_ijl]^k Mt_jl^k
// (moments of Sec. 2) collects, term by term and with the same truncation, into
//   u_i = sum_{||q|| <= p + 3} a^q W_i^q,
// where W depends on the cluster only (reg_stream).  The a^q follow the recurrence of
// the Taylor coefficients of (|d|^2 + eps^2)^(-nu) (recurrence_1 of the paper, which is
// the case nu = 1/2, eps = 0) at nu = -1/2:
//   n R^2 a^k = (2n - 3) sum_i d_i a^(k - e_i) - (n - 3) sum_i a^(k - 2e_i),  n = ||k||.
// One interaction thus costs one recurrence over nidx(p + 3) coefficients and three
// multiply-adds per coefficient, instead of three coefficient families and the
// product-rule contraction of every k.
#pragma once

#include "stk_math.hpp"

namespace stk {

// q! / (q - b)! per component (falling factorials), 0 if some q_m < b_m
STK_HD double falling(const int q[3], int b1, int b2, int b3) {
    const int b[3] = {b1, b2, b3};
    double r = 1.0;
    for (int m = 0; m < 3; ++m) {
        if (q[m] < b[m]) return 0.0;
        for (int s = 0; s < b[m]; ++s) r *= double(q[m] - s);
    }
    return r;
}

// Cluster stream of one multi-index q (||q|| <= p + 3): out[i] = W_i^q.  mom[a * ld + c]:
// c = 0..2 for M_c, c = 3 + 3j + l for Mt_jl, at graded-lex position a (||a|| <= p);
// moment indices outside ||k|| <= p vanish (the expansion is truncated at order p).
STK_HD void reg_stream(const double *mom, int ld, int p, const int q[3], double out[3]) {
    auto M = [&](int k1, int k2, int k3, int c) -> double {
        const int a = gidxp(k1, k2, k3, p);
        return a < 0 ? 0.0 : mom[a * ld + c];
    };
    auto tr = [&](int k1, int k2, int k3) -> double { return M(k1, k2, k3, 3) + M(k1, k2, k3, 7) + M(k1, k2, k3, 11); };
    for (int i = 0; i < 3; ++i) {
        const int ei[3] = {i == 0, i == 1, i == 2};
        double w = 0.0;
        for (int m = 0; m < 3; ++m) {
            const int em[3] = {m == 0, m == 1, m == 2};
            // S: delta_ij lap R, alpha = 2 e_m
            w += falling(q, 2 * em[0], 2 * em[1], 2 * em[2]) * M(q[0] - 2 * em[0], q[1] - 2 * em[1], q[2] - 2 * em[2], i);
            // S: -D_ij R, alpha = e_i + e_m (m plays j)
            w -= falling(q, ei[0] + em[0], ei[1] + em[1], ei[2] + em[2]) *
                 M(q[0] - ei[0] - em[0], q[1] - ei[1] - em[1], q[2] - ei[2] - em[2], m);
            // T: -(1/6) delta_jl D_i lap R = +(1/6) (alpha = e_i + 2 e_m) tr Mt
            {
                const int b[3] = {ei[0] + 2 * em[0], ei[1] + 2 * em[1], ei[2] + 2 * em[2]};
                w += falling(q, b[0], b[1], b[2]) / 6.0 * tr(q[0] - b[0], q[1] - b[1], q[2] - b[2]);
            }
            for (int l = 0; l < 3; ++l) {
                const int el[3] = {l == 0, l == 1, l == 2};
                // T: (1/3) D_ijl R, |alpha| = 3 (m plays j)
                const int b[3] = {ei[0] + em[0] + el[0], ei[1] + em[1] + el[1], ei[2] + em[2] + el[2]};
                w -= falling(q, b[0], b[1], b[2]) / 3.0 * M(q[0] - b[0], q[1] - b[1], q[2] - b[2], 3 + 3 * m + l);
                // T: -(1/6) (delta_ij D_l + delta_il D_j) lap R = +(1/6) (alpha = e_l + 2 e_m)
                //    (Mt_il + Mt_li)
                const int c[3] = {el[0] + 2 * em[0], el[1] + 2 * em[1], el[2] + 2 * em[2]};
                w += falling(q, c[0], c[1], c[2]) / 6.0 *
                     (M(q[0] - c[0], q[1] - c[1], q[2] - c[2], 3 + 3 * i + l) +
                      M(q[0] - c[0], q[1] - c[1], q[2] - c[2], 3 + 3 * l + i));
            }
        }
        out[i] = w;
    }
}

// Stream layout.  The kernel consumes the stream in the order it produces the a^q (graded
// lex, orders 2 .. p + 3; orders 0 and 1 have W = 0): W^q (3 values) per coefficient, and
// for the coefficients of order p + 1 also V^q = sum_j W^(q + 2e_j) right after it.  The
// top order's coefficients are needed by no later coefficient, so the grandparent term of
// their recurrence is contracted where the grandparents are made:
//   sum_{||q|| = p+3} a^q W^q = c1 sum_q s1(q) W^q - c2 sum_{||k|| = p+1} a^k V^k,
// with c1, c2 the factors of order p + 3; then order p + 3 reads order p + 2 only, and at
// most about |order p + 2| + |order p + 1| coefficients are live at once instead of
// |order p + 2| + |order p + 1| + part of order p + 3.  (For p = 0 the factor c2 of order 3
// is zero and no V is stored.)
STK_HD constexpr int reg_vorder(int p) { return p >= 1 ? p + 1 : -1; }
// stream position of the first value of the coefficient at graded-lex position a (-1 for
// orders 0 and 1)
STK_HD constexpr int reg_spos(int p, int a) {
    const int n = ordc(a), nv = reg_vorder(p);
    if (n < 2) return -1;
    int s = 3 * (a - nidx(1));
    if (nv >= 2 && n > nv) s += 3 * (nidx(nv) - nidx(nv - 1));
    if (n == nv) s += 3 * (a - nidx(nv - 1));
    return s;
}
STK_HD constexpr int reg_stream_len(int p) {
    const int nv = reg_vorder(p);
    return 3 * (nidx(p + 3) - nidx(1)) + (nv >= 2 ? 3 * (nidx(nv) - nidx(nv - 1)) : 0);
}
// the stream values of the coefficient at position a (||a|| <= p + 3): writes W^a, and V^a
// at order p + 1, at their positions in `stream`
STK_HD void reg_stream_fill(const double *mom, int ld, int p, int a, double *stream) {
    int q[3];
    kof(a, q);
    const int n = q[0] + q[1] + q[2];
    if (n < 2) return;
    double *o = stream + reg_spos(p, a);
    reg_stream(mom, ld, p, q, o);
    if (n == reg_vorder(p)) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 3; ++j) {
            int qj[3] = {q[0], q[1], q[2]};
            qj[j] += 2;
            double w[3];
            reg_stream(mom, ld, p, qj, w);
            v[0] += w[0];
            v[1] += w[1];
            v[2] += w[2];
        }
        o[3] = v[0];
        o[4] = v[1];
        o[5] = v[2];
    }
}

// Far field of one (target, cluster) pair: the recurrence of the a^q fused with the
// contraction, straight-line code generated at compile time for each order P (every a^q
// lives in a register).  The stream is wave-uniform and read with scalar loads in batches
// of at most BW values: each batch is requested one batch ahead and waited for once,
// after the batch before it has been used, so the loads overlap the arithmetic instead of
// stalling it one load at a time.  CAS: read the stream through the constant address
// space (the kernel stores doubles between interactions, which would otherwise turn its
// uniform loads into vector loads).
template <int P, bool CAS = false> struct RegEval {
    using Ptr = std::conditional_t<CAS, const STK_CONST_AS double *, const double *>;
    static constexpr int PB = P + 3;
    static constexpr int NB = nidx(PB);
    static constexpr int NV = reg_vorder(P);
    static constexpr int WS = reg_stream_len(P);
    static constexpr int BW = 18;

    STK_HD static constexpr int per(int n) { return n < 2 ? 0 : (n == NV ? 6 : 3); }
    STK_HD static constexpr int spos(int q) { return ordc(q) < 2 ? 0 : reg_spos(P, q); }
    // end of the batch that starts at coefficient q: as many coefficients as fit BW values
    STK_HD static constexpr int bend(int q) {
        int s = 0;
        while (q < NB && s + per(ordc(q)) <= BW) s += per(ordc(q++));
        return q;
    }
    STK_HD static constexpr int bstart(int q) { return ordc(q) < 2 ? 0 : reg_spos(P, q); }
    STK_HD static constexpr int blen(int q) { return q >= NB ? 0 : (bend(q) == NB ? WS : bstart(bend(q))) - bstart(q); }

    // coefficient at graded-lex position Q and its contraction with the batch buffer wb,
    // whose first value is stream position S0
    template <int Q, int QE, int S0>
    STK_HD static void steps(double (&a)[NB], const double d[3], double ir2, const double (&wb)[BW], double acc[3],
                             double acc2[3]) {
        constexpr int N = ordc(Q);
        constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = N - K1 - K2;
        // c1 sum_i d_i a^(k - e_i) with c1 folded into d (the same scaled d for the whole
        // order: the compiler forms it once) and sum_i a^(k - 2e_i), over the terms that
        // exist, each sum started from its first term (a literal 0 + x is not folded in IEEE
        // arithmetic)
        const double c1 = (double(2 * N - 3) / double(N)) * ir2;
        const double e[3] = {c1 * d[0], c1 * d[1], c1 * d[2]};
        double s1;
        if constexpr (K1 > 0) {
            s1 = e[0] * a[gidx(K1 - 1, K2, K3)];
            if constexpr (K2 > 0) s1 += e[1] * a[gidx(K1, K2 - 1, K3)];
            if constexpr (K3 > 0) s1 += e[2] * a[gidx(K1, K2, K3 - 1)];
        } else if constexpr (K2 > 0) {
            s1 = e[1] * a[gidx(K1, K2 - 1, K3)];
            if constexpr (K3 > 0) s1 += e[2] * a[gidx(K1, K2, K3 - 1)];
        } else {
            s1 = e[2] * a[gidx(K1, K2, K3 - 1)];
        }
        constexpr bool HAS2 = (K1 > 1 || K2 > 1 || K3 > 1) && N != 3 && N != PB;
        if constexpr (HAS2) {
            const double c2 = (double(N - 3) / double(N)) * ir2;
            double s2;
            if constexpr (K1 > 1) {
                s2 = a[gidx(K1 - 2, K2, K3)];
                if constexpr (K2 > 1) s2 += a[gidx(K1, K2 - 2, K3)];
                if constexpr (K3 > 1) s2 += a[gidx(K1, K2, K3 - 2)];
            } else if constexpr (K2 > 1) {
                s2 = a[gidx(K1, K2 - 2, K3)];
                if constexpr (K3 > 1) s2 += a[gidx(K1, K2, K3 - 2)];
            } else {
                s2 = a[gidx(K1, K2, K3 - 2)];
            }
            a[Q] = s1 - c2 * s2;
        } else {
            a[Q] = s1;
        }
        if constexpr (N >= 2) {
            constexpr int O = spos(Q) - S0;
            acc[0] += a[Q] * wb[O];
            acc[1] += a[Q] * wb[O + 1];
            acc[2] += a[Q] * wb[O + 2];
            if constexpr (N == NV) {
                acc2[0] += a[Q] * wb[O + 3];
                acc2[1] += a[Q] * wb[O + 4];
                acc2[2] += a[Q] * wb[O + 5];
            }
        }
        if constexpr (Q + 1 < QE) steps<Q + 1, QE, S0>(a, d, ir2, wb, acc, acc2);
    }

    // the values are in registers from here on: waits for their loads (issued a batch
    // earlier) before the next batch's loads are issued
    STK_HD static void settle(double (&w)[BW]) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
        for (int j = 0; j < BW; j += 3) asm volatile("" : "+s"(w[j]), "+s"(w[j + 1]), "+s"(w[j + 2]));
#else
        (void)w;
#endif
    }
    STK_HD static void sched_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
        __builtin_amdgcn_sched_barrier(0);
#endif
    }

    template <int Q>
    STK_HD static void batch(double (&a)[NB], const double d[3], double ir2, Ptr __restrict__ W, double (&cur)[BW],
                             double acc[3], double acc2[3]) {
        constexpr int QE = bend(Q);
        double nxt[BW];
        if constexpr (QE < NB) {
            constexpr int S1 = bstart(QE), L1 = blen(QE);
#pragma unroll
            for (int j = 0; j < BW; ++j) nxt[j] = j < L1 ? W[S1 + j] : 0.0;
            sched_fence();
        }
        steps<Q, QE, bstart(Q)>(a, d, ir2, cur, acc, acc2);
        if constexpr (QE < NB) {
            settle(nxt);
            sched_fence();
            batch<QE>(a, d, ir2, W, nxt, acc, acc2);
        }
    }

    // d = x - y_c, R2 = |d|^2 + eps^2 > 0, W: the cluster's stream.  acc = u.
    STK_HD static void run(const double d[3], double R2, Ptr __restrict__ W, double acc[3]) {
        double a[NB];
        const double ir2 = 1.0 / R2;
        a[0] = sqrt(R2);
        double acc2[3] = {0.0, 0.0, 0.0};
        acc[0] = acc[1] = acc[2] = 0.0;
        double first[BW];
        constexpr int L0 = blen(1);
#pragma unroll
        for (int j = 0; j < BW; ++j) first[j] = j < L0 ? W[j] : 0.0;
        settle(first);
        batch<1>(a, d, ir2, W, first, acc, acc2);
        if constexpr (NV >= 2) {
            const double c2 = (double(PB - 3) / double(PB)) * ir2;
            acc[0] -= c2 * acc2[0];
            acc[1] -= c2 * acc2[1];
            acc[2] -= c2 * acc2[2];
        }
    }
};

}  // namespace stk
