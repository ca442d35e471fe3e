// Arithmetic of the particle-cluster far field, shared by the device kernels (and
// compiled for the host only by the unit check of this header).
//
// Notation of Wang, Tlupova & Krasny (arXiv 1811.12498): b^q are the Taylor
// coefficients of the Coulomb potential 1/|x - y| about the cluster centre
// (eq. GreenFunc), obtained from recurrence_1; M_j^k and Mt_jl^k are the cluster
// moments of Sec. 2; the far field is eq. S_final plus eq. T_final.
//
// Both S_final and T_final are linear in the moments and in d = x - y_c.  Collecting
// every term by the index q of the b it multiplies gives
//
//     u_i = sum_q b^q G_i^q + sum_l d_l sum_q b^q F_il^q ,     ||q|| <= p + 2,
//
// where G and F depend on the cluster only and are a fixed sparse linear map of the
// moments (phi_channels below).  F factors further (phi_ge), leaving 3 G and 3 E
// values per multi-index of order <= p + 1, so an interaction costs about 9 multiply-
// adds per multi-index on top of the recurrence, instead of forming sigma, tau, m,
// m_ij per k.
//
// Scaling.  With R = |d|, dh = d / R, t = rho / R (rho a power of two >= r, the
// cluster radius) the recurrence is run on bt^q = t^||q|| R^(||q||+1) b^q:
//     bt^0 = 1,  bt^k = c1_n sum_i dh_i bt^{k-e_i} - c2_n sum_i bt^{k-2e_i},
//     c1_n = (2n-1)/n * t,  c2_n = (n-1)/n * t^2,  n = ||k||,
// which is recurrence_1 divided through by R^(n+1) and multiplied by t^n.  With the
// cluster blocks stored as G^q / rho^||q|| and E^k / rho^(||k||+1), every bt^q is O(1)
// (t <= 2 theta), so FP32 neither overflows at small R nor underflows at small rho.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stk {

#define STK_HD __host__ __device__ __attribute__((always_inline)) inline

// number of multi-indices with ||k|| <= p
STK_HD constexpr int nidx(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// position of k in graded-lex order (n = 0..; k1 = n..0; k2 = n-k1..0), -1 if any
// component is negative
STK_HD constexpr int gidx(int k1, int k2, int k3) {
    return (k1 < 0 || k2 < 0 || k3 < 0)
               ? -1
               : (k1 + k2 + k3) * (k1 + k2 + k3 + 1) * (k1 + k2 + k3 + 2) / 6 +
                     (k2 + k3) * (k2 + k3 + 1) / 2 + k3;
}

// order, first and second component of the multi-index at graded-lex position a
// (compile-time forms of kof)
STK_HD constexpr int ordc(int a) {
    int n = 0;
    while (nidx(n) <= a) ++n;
    return n;
}
STK_HD constexpr int kof1c(int a) {
    const int n = ordc(a);
    int r = a - (n > 0 ? nidx(n - 1) : 0), k1 = n;
    while (r >= n - k1 + 1) {
        r -= n - k1 + 1;
        --k1;
    }
    return k1;
}
STK_HD constexpr int kof2c(int a) {
    const int n = ordc(a);
    int r = a - (n > 0 ? nidx(n - 1) : 0), k1 = n;
    while (r >= n - k1 + 1) {
        r -= n - k1 + 1;
        --k1;
    }
    return n - k1 - r;
}

// gidx restricted to ||k|| <= p
STK_HD constexpr int gidxp(int k1, int k2, int k3, int p) {
    return (k1 + k2 + k3 > p) ? -1 : gidx(k1, k2, k3);
}

// multi-index of position a (inverse of gidx)
STK_HD void kof(int a, int k[3]) {
    int n = 0;
    while (nidx(n) <= a) ++n;
    int r = a - (n > 0 ? nidx(n - 1) : 0);
    // within order n: k1 = n..0, each k1 has (n - k1 + 1) entries
    int k1 = n;
    while (r >= n - k1 + 1) {
        r -= n - k1 + 1;
        --k1;
    }
    k[0] = k1;
    k[1] = n - k1 - r;
    k[2] = r;
}

// Moments of one cluster and one right-hand side: mom[a * ld + c], c = 0..2 for M_c,
// c = 3 + 3j + l for Mt_jl.  Returns the 12 channels of W^q for multi-index q
// (||q|| <= p + 2): out[i] = G_i^q, out[3 + 3i + l] = F_il^q.  Terms whose moment
// index falls outside ||k|| <= p vanish (the expansion is truncated at order p).
STK_HD void phi_channels(const double *mom, int ld, int p, const int q[3], double out[12]) {
    auto M = [&](int k1, int k2, int k3, int c) -> double {
        const int a = gidxp(k1, k2, k3, p);
        return a < 0 ? 0.0 : mom[a * ld + c];
    };
    for (int c = 0; c < 12; ++c) out[c] = 0.0;
    for (int i = 0; i < 3; ++i) {
        int ei[3] = {i == 0, i == 1, i == 2};
        double G = 0.0;
        // S_final: 2 b^k M_i^k
        G += 2.0 * M(q[0], q[1], q[2], i);
        for (int j = 0; j < 3; ++j) {
            int ej[3] = {j == 0, j == 1, j == 2};
            // S_final: -(k_i+1) b^{k+e_i-e_j} M_j^k, k = q - e_i + e_j
            G -= (q[i] + (i == j)) * M(q[0] - ei[0] + ej[0], q[1] - ei[1] + ej[1], q[2] - ei[2] + ej[2], j);
            // T_final: (k_j+1) b^{k+e_j} m_ij^k, k = q - e_j
            {
                const int k1 = q[0] - ej[0], k2 = q[1] - ej[1], k3 = q[2] - ej[2];
                G += q[j] / 3.0 * (M(k1, k2, k3, 3 + 3 * i + j) + M(k1, k2, k3, 3 + 3 * j + i));
            }
            for (int l = 0; l < 3; ++l) {
                int el[3] = {l == 0, l == 1, l == 2};
                // T_final: -(k_i+1)(k_j+1+delta_ij) b^{k+e_i+e_j-e_l} Mt_jl^k
                const int k[3] = {q[0] - ei[0] - ej[0] + el[0], q[1] - ei[1] - ej[1] + el[1],
                                  q[2] - ei[2] - ej[2] + el[2]};
                G -= (k[i] + 1) * (k[j] + 1 + (i == j)) / 3.0 * M(k[0], k[1], k[2], 3 + 3 * j + l);
            }
        }
        // T_final: (k_i+1) b^{k+e_i} m^k, k = q - e_i
        {
            const int k1 = q[0] - ei[0], k2 = q[1] - ei[1], k3 = q[2] - ei[2];
            G += q[i] / 3.0 * (M(k1, k2, k3, 3) + M(k1, k2, k3, 7) + M(k1, k2, k3, 11));
        }
        out[i] = G;
        for (int l = 0; l < 3; ++l) {
            // S_final: (k_i+1) b^{k+e_i} d_l M_l^k, k = q - e_i
            double F = q[i] * M(q[0] - ei[0], q[1] - ei[1], q[2] - ei[2], l);
            // T_final: (k_i+1)(k_j+1+delta_ij) b^{k+e_i+e_j} d_l Mt_jl^k, k = q - e_i - e_j
            for (int j = 0; j < 3; ++j) {
                int ej[3] = {j == 0, j == 1, j == 2};
                F += q[i] * (q[j] - (i == j)) / 3.0 *
                     M(q[0] - ei[0] - ej[0], q[1] - ei[1] - ej[1], q[2] - ei[2] - ej[2], 3 + 3 * j + l);
            }
            out[3 + 3 * i + l] = F;
        }
    }
}

// The F channels factor: F_il^q = q_i E_l^{q-e_i} with
//     E_l^k = M_l^k + (1/3) sum_j k_j Mt_jl^{k-e_j},     ||k|| <= p + 1,
// (substitute k = q - e_i in the two F terms above), so the F part of the far field is
//     sum_l d_l sum_q b^q F_il^q = sum_k (k_i + 1) b^{k+e_i} (d . E^k).
// G vanishes for ||q|| = p + 2.  A cluster therefore needs 3 G and 3 E values per
// multi-index of order <= p + 1.  Returns G^a (out[0..2]) and E^a (out[3..5]).
STK_HD void phi_ge(const double *mom, int ld, int p, const int a3[3], double out[6]) {
    double ch[12];
    phi_channels(mom, ld, p, a3, ch);
    out[0] = ch[0];
    out[1] = ch[1];
    out[2] = ch[2];
    auto M = [&](int k1, int k2, int k3, int c) -> double {
        const int a = gidxp(k1, k2, k3, p);
        return a < 0 ? 0.0 : mom[a * ld + c];
    };
    for (int l = 0; l < 3; ++l) {
        double e = M(a3[0], a3[1], a3[2], l);
        e += a3[0] / 3.0 * M(a3[0] - 1, a3[1], a3[2], 3 + l);
        e += a3[1] / 3.0 * M(a3[0], a3[1] - 1, a3[2], 6 + l);
        e += a3[2] / 3.0 * M(a3[0], a3[1], a3[2] - 1, 9 + l);
        out[3 + l] = e;
    }
}

// ---------------------------------------------------------------------------------
// Far field of one (target, cluster) pair: the scaled recurrence fused with the G/E
// contraction, as straight-line code generated at compile time for each order P (every
// b^q lives in a register).
//
// G = 1/|x - y| is harmonic in y, so for every multi-index m
//     sum_i (m_i + 1)(m_i + 2) b^{m + 2e_i} = 0.
// Taking m = k - 2e_3 gives, for k_3 >= 2,
//     k_3 (k_3 - 1) b^k = -(k_1 + 1)(k_1 + 2) b^{k + 2e_1 - 2e_3} - (k_2 + 1)(k_2 + 2) b^{k + 2e_2 - 2e_3},
// two coefficients of the same order (the relation is homogeneous in the order, so it
// holds for the scaled bt too).  recurrence_1 is therefore run only for the layers
// k_3 = 0 and k_3 = 1, which read only those two layers of the two orders below; the
// other layers are filled from the harmonic relation.  Within an order the layers are
// produced in increasing k_3, and the E contraction of layer j of the previous order
// runs as soon as layers j and j + 1 exist, so few coefficients are live at once.
//
// Cluster block ("stream"): G^0, then for n = 1 .. P + 2 and layer j = 0 .. n the chunk
//   [ G^q for q of order n, k_3 = j   (if n <= P + 1) ]
//   [ E^k for k of order n - 1, k_3 = j - 1   (if j >= 1) ]
// with entries in decreasing k_1, three values each: the order in which the kernel
// consumes them, so each chunk is one contiguous scalar-cache read.  Values are stored
// as G^q / rho^||q|| and E^k / rho^(||k||+1).  Total 6 nidx(P + 1) values.
// ---------------------------------------------------------------------------------
STK_HD constexpr int stream_gpart(int p, int n, int j) { return n <= p + 1 ? 3 * (n - j + 1) : 0; }
STK_HD constexpr int stream_epart(int n, int j) { return j >= 1 ? 3 * (n - j + 1) : 0; }
STK_HD constexpr int stream_off(int p, int n, int j) {
    int o = 3;
    for (int m = 1; m < n; ++m)
        for (int jj = 0; jj <= m; ++jj) o += stream_gpart(p, m, jj) + stream_epart(m, jj);
    for (int jj = 0; jj < j; ++jj) o += stream_gpart(p, n, jj) + stream_epart(n, jj);
    return o;
}
// stream positions of G^a and E^a for multi-index a (||a|| <= p + 1)
STK_HD void stream_pos(int p, const int a[3], int &g, int &e) {
    const int n = a[0] + a[1] + a[2], j = a[2], i = (n - j) - a[0];
    g = n == 0 ? 0 : stream_off(p, n, j) + 3 * i;
    e = stream_off(p, n + 1, j + 1) + stream_gpart(p, n + 1, j + 1) + 3 * i;
}

// KB right-hand sides share one recurrence: their streams follow each other at a
// stride of WS values and each has its own pair of partial sums
// read-only device data that no store of the running kernel can touch, read through the
// constant address space: loads at wave-uniform addresses then stay scalar even where the
// kernel stores elsewhere in between (the host build of the same code sees plain pointers)
#if defined(__HIP_DEVICE_COMPILE__)
#define STK_CONST_AS __attribute__((address_space(4)))
#else
#define STK_CONST_AS
#endif

// CAS: read the streams through the constant address space (needed where the kernel
// stores values of the stream's own type between interactions)
template <int P, typename T, int KB = 1, bool CAS = false> struct FarEval {
    using Ptr = std::conditional_t<CAS, const STK_CONST_AS T *, const T *>;
    static constexpr int PB = P + 2;
    static constexpr int NB = nidx(PB);
    static constexpr int WS = 6 * nidx(P + 1);

    template <int N, int I> STK_HD static void gterm(T bq, Ptr __restrict__ G, T (*accG)[3]) {
        if constexpr (N <= P + 1) {
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                accG[r][0] += bq * G[r * WS + 3 * I];
                accG[r][1] += bq * G[r * WS + 3 * I + 1];
                accG[r][2] += bq * G[r * WS + 3 * I + 2];
            }
        }
    }

    // all coefficients of order N in layer K3 (k1 = N - K3 .. 0), with their G terms;
    // G points at the chunk (N, K3).  e = c1 dh (the order's first factor folded into the
    // direction, once per order); the recurrence's sums start from their first term (a
    // literal 0 + x is not folded in IEEE arithmetic).
    template <int N, int K3, int K1>
    STK_HD static void layer(T (&b)[NB], const T e[3], T c2, Ptr __restrict__ G, T (*accG)[3]) {
        constexpr int K2 = N - K3 - K1;
        constexpr int Q = gidx(K1, K2, K3);
        if constexpr (K3 <= 1) {  // recurrence_1, scaled
            T s1;
            if constexpr (K1 > 0) {
                s1 = e[0] * b[gidx(K1 - 1, K2, K3)];
                if constexpr (K2 > 0) s1 += e[1] * b[gidx(K1, K2 - 1, K3)];
                if constexpr (K3 > 0) s1 += e[2] * b[gidx(K1, K2, K3 - 1)];
            } else if constexpr (K2 > 0) {
                s1 = e[1] * b[gidx(K1, K2 - 1, K3)];
                if constexpr (K3 > 0) s1 += e[2] * b[gidx(K1, K2, K3 - 1)];
            } else {
                s1 = e[2] * b[gidx(K1, K2, K3 - 1)];
            }
            if constexpr (N > 1 && (K1 > 1 || K2 > 1)) {
                T s2;
                if constexpr (K1 > 1) {
                    s2 = b[gidx(K1 - 2, K2, K3)];
                    if constexpr (K2 > 1) s2 += b[gidx(K1, K2 - 2, K3)];
                } else {
                    s2 = b[gidx(K1, K2 - 2, K3)];
                }
                b[Q] = s1 - c2 * s2;
            } else {
                b[Q] = s1;
            }
        } else {  // harmonic fill
            constexpr double den = double(K3 * (K3 - 1));
            constexpr double ca = -double((K1 + 1) * (K1 + 2)) / den;
            constexpr double cb = -double((K2 + 1) * (K2 + 2)) / den;
            b[Q] = T(ca) * b[gidx(K1 + 2, K2, K3 - 2)] + T(cb) * b[gidx(K1, K2 + 2, K3 - 2)];
        }
        gterm<N, (N - K3) - K1>(b[Q], G, accG);
        if constexpr (K1 > 0) layer<N, K3, K1 - 1>(b, e, c2, G, accG);
    }

    // E contraction for the k of order N - 1 in layer K3 (needs layers K3, K3 + 1 of
    // order N); E points at the E part of chunk (N, K3 + 1).  The third component's
    // factor k_3 + 1 is the same for the whole layer: its terms go to acc3 unscaled and
    // the caller applies the factor once.
    template <int N, int K3, int K1>
    STK_HD static void elayer(const T (&b)[NB], const T dh[3], Ptr __restrict__ E, T (*accF)[3], T *acc3) {
        constexpr int M = N - 1;
        constexpr int K2 = M - K3 - K1;
        constexpr int I = (M - K3) - K1;
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            Ptr __restrict__ Er = E + r * WS;
            const T sig = dh[0] * Er[3 * I] + dh[1] * Er[3 * I + 1] + dh[2] * Er[3 * I + 2];
            accF[r][0] += b[gidx(K1 + 1, K2, K3)] * (T(K1 + 1) * sig);
            accF[r][1] += b[gidx(K1, K2 + 1, K3)] * (T(K2 + 1) * sig);
            acc3[r] += b[gidx(K1, K2, K3 + 1)] * sig;
        }
        if constexpr (K1 > 0) elayer<N, K3, K1 - 1>(b, dh, E, accF, acc3);
    }

    // returns 0 through an asm the optimiser cannot see into.  Adding it to the block
    // pointer pins each chunk's scalar loads after the previous chunk's accumulations,
    // instead of letting every load of the interaction be hoisted to the top (they do
    // not fit in SGPRs); the asm touches no memory, so the loads stay scalar.
    STK_HD static int fence(T dep) {
        int z = 0;
#if defined(__HIP_DEVICE_COMPILE__)
        asm("" : "+s"(z) : "v"(dep));
        z = __builtin_amdgcn_readfirstlane(z);
#else
        (void)dep;
#endif
        return z;
    }

    template <int N, int J>
    STK_HD static void layers_from(T (&b)[NB], const T dh[3], const T e[3], T c2, Ptr __restrict__ W,
                                   T (*accG)[3], T (*accF)[3]) {
        if constexpr (J <= N) {
            Ptr __restrict__ chunk = W + stream_off(P, N, J) + fence(accG[0][0] + accF[0][0]);
            layer<N, J, N - J>(b, e, c2, chunk, accG);
            if constexpr (J == 1) {  // layer k_3 = 0: factor 1
                T acc3[KB];
#pragma unroll
                for (int r = 0; r < KB; ++r) acc3[r] = accF[r][2];
                elayer<N, 0, N - 1>(b, dh, chunk + stream_gpart(P, N, J), accF, acc3);
#pragma unroll
                for (int r = 0; r < KB; ++r) accF[r][2] = acc3[r];
            } else if constexpr (J >= 2) {
                T acc3[KB];
#pragma unroll
                for (int r = 0; r < KB; ++r) acc3[r] = T(0);
                elayer<N, J - 1, N - J>(b, dh, chunk + stream_gpart(P, N, J), accF, acc3);
#pragma unroll
                for (int r = 0; r < KB; ++r) accF[r][2] += T(J) * acc3[r];
            }
            layers_from<N, J + 1>(b, dh, e, c2, W, accG, accF);
        }
    }

    template <int N>
    STK_HD static void order(T (&b)[NB], const T dh[3], T t, Ptr __restrict__ W, T (*accG)[3], T (*accF)[3]) {
        const T c1 = T(2 * N - 1) / T(N) * t;
        const T c2 = T(N - 1) / T(N) * (t * t);
        const T e[3] = {c1 * dh[0], c1 * dh[1], c1 * dh[2]};
        layers_from<N, 0>(b, dh, e, c2, W, accG, accF);
        if constexpr (N < PB) order<N + 1>(b, dh, t, W, accG, accF);
    }

    // W: the first right-hand side's cluster stream.  u_i = accG[r][i] / R + accF[r][i]
    STK_HD static void run(const T dh[3], T t, Ptr __restrict__ W, T (*accG)[3], T (*accF)[3]) {
        T b[NB];
        b[0] = T(1);
#pragma unroll
        for (int r = 0; r < KB; ++r) {
            accG[r][0] = W[r * WS];
            accG[r][1] = W[r * WS + 1];
            accG[r][2] = W[r * WS + 2];
            accF[r][0] = accF[r][1] = accF[r][2] = T(0);
        }
        order<1>(b, dh, t, W, accG, accF);
    }
    // one right-hand side
    STK_HD static void run(const T dh[3], T t, Ptr __restrict__ W, T accG[3], T accF[3]) {
        run(dh, t, W, reinterpret_cast<T(*)[3]>(accG), reinterpret_cast<T(*)[3]>(accF));
    }
};

// velocity of one far interaction from the two partial sums
template <typename T> STK_HD void far_velocity(const T accG[3], const T accF[3], T rinv, T u[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) u[i] = accG[i] * rinv + accF[i];
}

// power of two >= r (1 when r == 0): the per-cluster scale of the channel blocks
STK_HD double rho_of(double r) {
    if (!(r > 0.0)) return 1.0;
    int e;
    const double m = frexp(r, &e);  // r = m * 2^e, m in [0.5, 1)
    return ldexp(1.0, m == 0.5 ? e - 1 : e);
}

// Neumaier-compensated accumulator
template <typename T> struct Comp {
    T s = T(0), c = T(0);
    STK_HD void add(T v) {
        const T t = s + v;
        if (fabs(s) >= fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    STK_HD double value() const { return double(s) + double(c); }
};

}  // namespace stk
