// Far-field adjoint kernels (the transpose of the frozen-plan treecode operator).
//
// For L = sum_m w^m . u^m with the interaction lists, cluster centres and scales held
// fixed, one far interaction contributes (stk_math.hpp notation, scaled quantities)
//     L_mC = sum_q (w . Ghat^q) bt^q / R + sum_k (dh . Ehat^k) zh^k,
//     zh^k = sum_i w_i (k_i + 1) bt^{k + e_i},
// which is linear in the cluster stream (Ghat, Ehat).  Two kernels use it:
//   k_far_lambda  accumulates dL/dGhat_i^q = sum_m (w_i / R) bt^q and
//                 dL/dEhat_l^k = sum_m dh_l zh^k over the targets that accept the cluster
//                 (cluster-major work items; per order the wave writes its targets'
//                 coefficients to LDS and each lane sums whole columns);
//   k_far_tgrad   dL/dx for each target, from d/dx_s b^q = -(q_s + 1) b^{q + e_s}:
//     dL/dx_s = -(1/(R rho)) sum_q (q_s+1) bt^{q+e_s} (w . Ghat^q)
//               -(1/rho) sum_k (dh . Ehat^k) sum_i w_i (k_i+1)(k_s+1+delta_is) bt^{k+e_i+e_s}
//               +(1/R) sum_k Ehat_s^k zh^k,
//     which needs coefficients up to order p + 3.
#pragma once

#include "far_kernels.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {

// ---------------------------------------------------------------------------------
// coefficients bt^q of one (target, cluster) pair up to order PB in registers: the
// scaled recurrence_1 for layers k3 <= 1 and the harmonic fill for k3 >= 2 (the same
// arithmetic as FarEval), calling Visit::coef<Q, N>(bq) as each coefficient is formed
// and Visit::order_done<N>(b) after each order
// ---------------------------------------------------------------------------------
template <int PB, typename T, class Visit> struct Coefs {
    static constexpr int NB = nidx(PB);

    template <int N, int K3, int K1> STK_HD static void layer(T (&b)[NB], const T dh[3], T c1, T c2, Visit &v) {
        constexpr int K2 = N - K3 - K1;
        constexpr int Q = gidx(K1, K2, K3);
        if constexpr (K3 <= 1) {
            T s1 = T(0), s2 = T(0);
            if constexpr (K1 > 0) s1 += dh[0] * b[gidx(K1 - 1, K2, K3)];
            if constexpr (K2 > 0) s1 += dh[1] * b[gidx(K1, K2 - 1, K3)];
            if constexpr (K3 > 0) s1 += dh[2] * b[gidx(K1, K2, K3 - 1)];
            if constexpr (K1 > 1) s2 += b[gidx(K1 - 2, K2, K3)];
            if constexpr (K2 > 1) s2 += b[gidx(K1, K2 - 2, K3)];
            if constexpr (N > 1)
                b[Q] = c1 * s1 - c2 * s2;
            else
                b[Q] = c1 * s1;
        } else {
            constexpr double den = double(K3 * (K3 - 1));
            constexpr double ca = -double((K1 + 1) * (K1 + 2)) / den;
            constexpr double cb = -double((K2 + 1) * (K2 + 2)) / den;
            b[Q] = T(ca) * b[gidx(K1 + 2, K2, K3 - 2)] + T(cb) * b[gidx(K1, K2 + 2, K3 - 2)];
        }
        v.template coef<Q, N>(b[Q]);
        if constexpr (K1 > 0) layer<N, K3, K1 - 1>(b, dh, c1, c2, v);
    }

    template <int N, int J> STK_HD static void layers(T (&b)[NB], const T dh[3], T c1, T c2, Visit &v) {
        if constexpr (J <= N) {
            layer<N, J, N - J>(b, dh, c1, c2, v);
            layers<N, J + 1>(b, dh, c1, c2, v);
        }
    }

    template <int N> STK_HD static void order(T (&b)[NB], const T dh[3], T t, Visit &v) {
        const T c1 = T(2 * N - 1) / T(N) * t;
        const T c2 = T(N - 1) / T(N) * (t * t);
        layers<N, 0>(b, dh, c1, c2, v);
        v.template order_done<N>(b);
        if constexpr (N < PB) order<N + 1>(b, dh, t, v);
    }

    STK_HD static void run(T (&b)[NB], const T dh[3], T t, Visit &v) {
        b[0] = T(1);
        v.template coef<0, 0>(b[0]);
        v.template order_done<0>(b);
        order<1>(b, dh, t, v);
    }
};

// ---------------------------------------------------------------------------------
// k_far_lambda
// ---------------------------------------------------------------------------------
struct LambdaArgs {
    const double *tpos;        // sorted targets
    const double *ws;          // sorted adjoint seed w (m,3)
    int64_t m;
    const int32_t *item_node;  // work item -> cluster
    const int32_t *item_e0;    // work item -> first position in the cluster-sorted entry list
    const int32_t *item_e1;
    const int32_t *ent;        // cluster-sorted far entries (indices into the group lists)
    const int32_t *ent_group;  // far entry -> group
    const uint64_t *mask;      // far entry -> lane mask
    const double *center, *rho;
    const int32_t *colpos;     // (orders, 2, LAM_ROW): stream position of each LDS column
    double *lambda;            // (nn, 6 nG) adjoint of the cluster streams, accumulated
    int32_t nitems;
};

constexpr int LPITCH = 65;   // LDS row pitch (targets), padded against bank conflicts
constexpr int LAM_ROW = 128; // entries per row of the column -> stream position table

template <int P> __host__ __device__ constexpr int lam_ncol_g(int n) { return n <= P + 1 ? (n + 1) * (n + 2) / 2 : 0; }
template <int P> __host__ __device__ constexpr int lam_ncol_e(int n) { return n >= 1 ? n * (n + 1) / 2 : 0; }
template <int P> __host__ __device__ constexpr int lam_maxcol() {
    int m = 1;
    for (int n = 0; n <= P + 2; ++n) {
        if (lam_ncol_g<P>(n) > m) m = lam_ncol_g<P>(n);
        if (lam_ncol_e<P>(n) > m) m = lam_ncol_e<P>(n);
    }
    return m;
}
// LDS of one work item: the FP64 stream accumulator first (8-byte aligned), then the
// column table and the two weight tables
template <int P, typename T> __host__ __device__ constexpr size_t lam_lds_bytes() {
    return sizeof(double) * 6 * nidx(P + 1) + sizeof(T) * (size_t(lam_maxcol<P>()) * LPITCH + 6 * 64);
}

template <int P, typename T> struct LambdaVisit {
    T *cols;       // [col][LPITCH]
    const T *cw;   // [3][64] w_i / R per target (0 for lanes outside the mask)
    const T *dw;   // [3][64] dh_l per target (0 outside the mask)
    double *acc;   // [6 nG] LDS accumulator in stream order
    const int32_t *colpos;
    T wl[3];       // this lane's w
    int lane;

    template <int Q, int N> STK_HD void coef(T bq) {
        if constexpr (N <= P + 1) cols[(Q - (N > 0 ? nidx(N - 1) : 0)) * LPITCH + lane] = bq;
    }

    // reduce columns [0, nc) of the LDS table over the 64 targets with weights wt
    STK_HD void reduce(int nc, const T *wt, const int32_t *pos) {
        __syncthreads();
        for (int col = lane; col < nc; col += 64) {
            T a0 = T(0), a1 = T(0), a2 = T(0);
            const T *row = cols + col * LPITCH;
#pragma unroll 4
            for (int mm = 0; mm < 64; ++mm) {
                const T v = row[mm];
                a0 += wt[mm] * v;
                a1 += wt[64 + mm] * v;
                a2 += wt[128 + mm] * v;
            }
            const int p0 = pos[col];
            acc[p0] += double(a0);
            acc[p0 + 1] += double(a1);
            acc[p0 + 2] += double(a2);
        }
        __syncthreads();
    }

    template <int N> STK_HD void order_done(const T (&b)[nidx(P + 2)]) {
        // G columns of order N (already written by coef)
        if constexpr (N <= P + 1) reduce(lam_ncol_g<P>(N), cw, colpos + (2 * N) * LAM_ROW);
        // E columns: zh^k for k of order N - 1
        if constexpr (N >= 1) {
            constexpr int M = N - 1;
            ecol<N, M, 0>(b);
            reduce(lam_ncol_e<P>(N), dw, colpos + (2 * N + 1) * LAM_ROW);
        }
    }

    // zh^k = sum_i w_i (k_i+1) bt^{k+e_i} for every k of order M, in graded-lex order
    template <int N, int M, int A> STK_HD void ecol(const T (&b)[nidx(P + 2)]) {
        if constexpr (A < (M + 1) * (M + 2) / 2) {
            constexpr int Q = (M > 0 ? nidx(M - 1) : 0) + A;
            constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = M - K1 - K2;
            const T z = wl[0] * (T(K1 + 1) * b[gidx(K1 + 1, K2, K3)]) + wl[1] * (T(K2 + 1) * b[gidx(K1, K2 + 1, K3)]) +
                        wl[2] * (T(K3 + 1) * b[gidx(K1, K2, K3 + 1)]);
            cols[A * LPITCH + lane] = z;
            ecol<N, M, A + 1>(b);
        }
    }

};

template <int P, typename T> __global__ __launch_bounds__(64) void k_far_lambda(LambdaArgs a) {
    constexpr int NG = nidx(P + 1);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *acc = reinterpret_cast<double *>(lds_raw);
    T *cols = reinterpret_cast<T *>(acc + 6 * NG);
    T *cw = cols + lam_maxcol<P>() * LPITCH;
    T *dw = cw + 192;
    const int lane = threadIdx.x;
    const int32_t it = blockIdx.x;
    if (it >= a.nitems) return;
    const int32_t c = a.item_node[it];
    for (int q = lane; q < 6 * NG; q += 64) acc[q] = 0.0;
    const double c0 = a.center[3 * c], c1 = a.center[3 * c + 1], c2 = a.center[3 * c + 2];
    const double rho = a.rho[c];
    for (int32_t e = a.item_e0[it]; e < a.item_e1[it]; ++e) {
        const int32_t ent = a.ent[e];
        const int32_t g = a.ent_group[ent];
        const uint64_t mk = a.mask[ent];
        const int64_t t = int64_t(g) * 64 + lane;
        const bool in = ((mk >> lane) & 1ull) && t < a.m;
        T dh[3] = {T(1), T(0), T(0)}, tt = T(0), wl[3] = {T(0), T(0), T(0)}, ri = T(0);
        if (in) {
            const double d0 = a.tpos[3 * t] - c0, d1 = a.tpos[3 * t + 1] - c1, d2 = a.tpos[3 * t + 2] - c2;
            const double rinv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            dh[0] = T(d0 * rinv);
            dh[1] = T(d1 * rinv);
            dh[2] = T(d2 * rinv);
            tt = T(rho * rinv);
            ri = T(rinv);
            wl[0] = T(a.ws[3 * t]);
            wl[1] = T(a.ws[3 * t + 1]);
            wl[2] = T(a.ws[3 * t + 2]);
        }
        __syncthreads();
        for (int i = 0; i < 3; ++i) {
            cw[64 * i + lane] = wl[i] * ri;
            dw[64 * i + lane] = in ? dh[i] : T(0);
        }
        LambdaVisit<P, T> v{cols, cw, dw, acc, a.colpos, {wl[0], wl[1], wl[2]}, lane};
        T b[nidx(P + 2)];
        Coefs<P + 2, T, LambdaVisit<P, T>>::run(b, dh, tt, v);
    }
    __syncthreads();
    double *out = a.lambda + size_t(c) * 6 * NG;
    for (int q = lane; q < 6 * NG; q += 64) atomicAdd(out + q, acc[q]);
}

// ---------------------------------------------------------------------------------
// k_far_tgrad: dL/dx for every target from its far list
// ---------------------------------------------------------------------------------
template <int P, typename T> struct TgradVisit {
    const T *W;   // cluster stream
    T dh[3], wl[3];
    T a1[3], a2[3], a3[3];

    template <int Q, int N> STK_HD void coef(T) {}

    // at order N (coefficients 0..N exist):
    //  term 1 for q of order N-1 (<= P+1): (w.Ghat^q) (q_s+1) bt^{q+e_s}
    //  term 3 for k of order N-1 (<= P+1): Ehat_s^k zh^k
    //  term 2 for k of order N-2 (<= P+1): (dh.Ehat^k) sum_i w_i (k_i+1)(k_s+1+delta_is) bt^{k+e_i+e_s}
    template <int N> STK_HD void order_done(const T (&b)[nidx(P + 3)]) {
        // the fence pins this order's scalar loads after the previous order's sums
        const T *__restrict__ Wf = W + FarEval<P, T>::fence(a1[0] + a2[0] + a3[0]);
        if constexpr (N >= 1 && N - 1 <= P + 1) walk13<N - 1, 0>(b, Wf);
        if constexpr (N >= 2 && N - 2 <= P + 1) walk2<N - 2, 0>(b, Wf);
    }

    template <int M, int A> STK_HD void walk13(const T (&b)[nidx(P + 3)], const T *__restrict__ W) {
        if constexpr (A < (M + 1) * (M + 2) / 2) {
            constexpr int Q = (M > 0 ? nidx(M - 1) : 0) + A;
            constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = M - K1 - K2;
            constexpr int kk[3] = {K1, K2, K3};
            int pg = 0, pe = 0;
            stream_pos_c(kk, pg, pe);
            const T g = wl[0] * W[pg] + wl[1] * W[pg + 1] + wl[2] * W[pg + 2];
            const T bx = b[gidx(K1 + 1, K2, K3)], by = b[gidx(K1, K2 + 1, K3)], bz = b[gidx(K1, K2, K3 + 1)];
            a1[0] += g * (T(K1 + 1) * bx);
            a1[1] += g * (T(K2 + 1) * by);
            a1[2] += g * (T(K3 + 1) * bz);
            const T z = wl[0] * (T(K1 + 1) * bx) + wl[1] * (T(K2 + 1) * by) + wl[2] * (T(K3 + 1) * bz);
            a3[0] += W[pe] * z;
            a3[1] += W[pe + 1] * z;
            a3[2] += W[pe + 2] * z;
            walk13<M, A + 1>(b, W);
        }
    }

    template <int M, int A> STK_HD void walk2(const T (&b)[nidx(P + 3)], const T *__restrict__ W) {
        if constexpr (A < (M + 1) * (M + 2) / 2) {
            constexpr int Q = (M > 0 ? nidx(M - 1) : 0) + A;
            constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = M - K1 - K2;
            constexpr int kk[3] = {K1, K2, K3};
            int pg = 0, pe = 0;
            stream_pos_c(kk, pg, pe);
            const T sig = dh[0] * W[pe] + dh[1] * W[pe + 1] + dh[2] * W[pe + 2];
            // h_s = sum_i w_i (k_i+1)(k_s+1+delta_is) bt^{k+e_i+e_s}
            const T w0 = wl[0] * T(K1 + 1), w1 = wl[1] * T(K2 + 1), w2 = wl[2] * T(K3 + 1);
            const T hx = w0 * T(K1 + 2) * b[gidx(K1 + 2, K2, K3)] + w1 * T(K1 + 1) * b[gidx(K1 + 1, K2 + 1, K3)] +
                         w2 * T(K1 + 1) * b[gidx(K1 + 1, K2, K3 + 1)];
            const T hy = w0 * T(K2 + 1) * b[gidx(K1 + 1, K2 + 1, K3)] + w1 * T(K2 + 2) * b[gidx(K1, K2 + 2, K3)] +
                         w2 * T(K2 + 1) * b[gidx(K1, K2 + 1, K3 + 1)];
            const T hz = w0 * T(K3 + 1) * b[gidx(K1 + 1, K2, K3 + 1)] + w1 * T(K3 + 1) * b[gidx(K1, K2 + 1, K3 + 1)] +
                         w2 * T(K3 + 2) * b[gidx(K1, K2, K3 + 2)];
            a2[0] += sig * hx;
            a2[1] += sig * hy;
            a2[2] += sig * hz;
            walk2<M, A + 1>(b, W);
        }
    }

    STK_HD static constexpr void stream_pos_c(const int (&k)[3], int &g, int &e) {
        const int n = k[0] + k[1] + k[2], j = k[2], i = (n - j) - k[0];
        g = n == 0 ? 0 : stream_off(P, n, j) + 3 * i;
        e = stream_off(P, n + 1, j + 1) + stream_gpart(P, n + 1, j + 1) + 3 * i;
    }
};

struct TgradArgs {
    const double *tpos, *ws;
    int64_t m;
    const int32_t *off, *node;
    const uint64_t *mask;
    const double *center, *rho;
    const void *wblk;
    double *gt;   // (m,3) sorted order, written
    int32_t ngroups;
};

template <int P, typename T> __global__ __launch_bounds__(64) void k_far_tgrad(TgradArgs a) {
    constexpr int NG = nidx(P + 1);
    const int32_t g = xcd_group(a.ngroups);
    if (g >= a.ngroups) return;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    const bool valid = t < a.m;
    double x0 = 0, x1 = 0, x2 = 0, w0 = 0, w1 = 0, w2 = 0;
    if (valid) {
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
        w0 = a.ws[3 * t];
        w1 = a.ws[3 * t + 1];
        w2 = a.ws[3 * t + 2];
    }
    const T *wb = static_cast<const T *>(a.wblk);
    Comp<T> acc[3];
    for (int32_t e = a.off[g]; e < a.off[g + 1]; ++e) {
        const int32_t c = __builtin_amdgcn_readfirstlane(a.node[e]);
        const uint64_t mk = a.mask[e];
        if ((mk >> lane) & 1ull) {
            const double d0 = x0 - a.center[3 * c], d1 = x1 - a.center[3 * c + 1], d2 = x2 - a.center[3 * c + 2];
            const double rinv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const double rho = a.rho[c];
            TgradVisit<P, T> v{wb + size_t(c) * 6 * NG,
                               {T(d0 * rinv), T(d1 * rinv), T(d2 * rinv)},
                               {T(w0), T(w1), T(w2)},
                               {T(0), T(0), T(0)},
                               {T(0), T(0), T(0)},
                               {T(0), T(0), T(0)}};
            T b[nidx(P + 3)];
            Coefs<P + 3, T, TgradVisit<P, T>>::run(b, v.dh, T(rho * rinv), v);
            const T f1 = T(-rinv / rho), f2 = T(-1.0 / rho), f3 = T(rinv);
            for (int s = 0; s < 3; ++s) acc[s].add(f1 * v.a1[s] + f2 * v.a2[s] + f3 * v.a3[s]);
        }
    }
    if (valid) {
        a.gt[3 * t] = acc[0].value();
        a.gt[3 * t + 1] = acc[1].value();
        a.gt[3 * t + 2] = acc[2].value();
    }
}

template <int P, typename T> void launch_far_lambda(const LambdaArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    hipLaunchKernelGGL((k_far_lambda<P, T>), dim3(a.nitems), dim3(64), (lam_lds_bytes<P, T>()), s, a);
    STK_CHECK_LAUNCH();
}

template <int P, typename T> void launch_far_tgrad(const TgradArgs &a, hipStream_t s) {
    if (a.ngroups == 0) return;
    hipLaunchKernelGGL((k_far_tgrad<P, T>), dim3(xcd_blocks(a.ngroups)), dim3(64), 0, s, a);
    STK_CHECK_LAUNCH();
}

}  // namespace stk
