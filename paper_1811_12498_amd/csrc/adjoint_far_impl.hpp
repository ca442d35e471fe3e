// Far-field adjoint kernel bodies (instantiated per Taylor order in adj_p*.hip and
// adjt_p*.hip); the operator they apply is described in adjoint_far.hpp.
#pragma once

#include "adjoint_far.hpp"

namespace stk {

// ---------------------------------------------------------------------------------
// coefficients bt^q of one (target, cluster) pair up to order PB in registers: the
// scaled recurrence_1 for layers k3 <= 1 and the harmonic fill for k3 >= 2 (the same
// arithmetic as FarEval), calling Visit::coef<Q, N>(bq) as each coefficient is formed,
// Visit::layer_done<N, J>(b) after layer k3 = J of order N and Visit::order_done<N>(b)
// after each order
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
            v.template layer_done<N, J>(b);
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

// x + (x of lane ^ o) in every lane, o = 16 or 32, through the VALU's lane-half swaps (the
// two outputs of a swap of x with itself hold x and its partner in opposite halves, so their
// sum is the pair sum whatever the orientation)
STK_HD float pair_sum(float x, int o) {
#if defined(__HIP_DEVICE_COMPILE__)
    const unsigned u = __float_as_uint(x);
    const auto r = o == 32 ? __builtin_amdgcn_permlane32_swap(u, u, false, false)
                           : __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
#else
    return x + __shfl_xor(x, o);
#endif
}
STK_HD double pair_sum(double x, int o) {
#if defined(__HIP_DEVICE_COMPILE__)
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = unsigned(b), hi = unsigned(b >> 32);
    const auto l = o == 32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                           : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = o == 32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                           : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    const double x0 = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[0]) << 32) | l[0]));
    const double x1 = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(h[1]) << 32) | l[1]));
    return x0 + x1;
#else
    return x + __shfl_xor(x, o);
#endif
}

template <int P, typename T> struct LambdaVisit {
    static constexpr int NCOL = lam_ncol(P);
    static constexpr int TBL = lam_tbl<T>(), WP = lam_wp<T>();
    static constexpr int PITCH = lam_pitch<T>(), NV = lam_nv<T>();
    using V = std::conditional_t<sizeof(T) == 4, float4, double2>;  // one 16-byte LDS read
    T *cols;       // [TBL][PITCH]: the current batch
    const T *cw;   // [3][WP] w_i / R per target (0 for idle lanes), at lam_wid(target)
    const T *dw;   // [3][WP] dh_l per target (0 for idle lanes)
    T *acc;        // [6 nG] LDS accumulator in stream order
    const int32_t *cpos, *ckind;
    T wl[3];       // this lane's w
    int lane;

    // reduce the nc columns of batch bt over the 64 targets: lane = (column, run of
    // TBL targets), the runs' sums combined across lanes
    STK_HD void reduce(int nc, int bt) {
        __syncthreads();
        const int col = lane % TBL, run = lane / TBL, t0 = run * TBL;
        const bool on = col < nc;
        T a0 = T(0), a1 = T(0), a2 = T(0);
        int p0 = 0;
        if (on) {
            const int c = bt * TBL + col;
            p0 = cpos[c];
            // rows and weight runs are 16-byte aligned: NV values per LDS read
            const T *wt = (ckind[c] ? dw : cw) + lam_wid<T>(t0);
            const T *row = cols + col * PITCH + t0;
#pragma unroll 2
            for (int mm = 0; mm < TBL; mm += NV) {
                const V rv = *reinterpret_cast<const V *>(row + mm);
                const V w0 = *reinterpret_cast<const V *>(wt + mm);
                const V w1 = *reinterpret_cast<const V *>(wt + WP + mm);
                const V w2 = *reinterpret_cast<const V *>(wt + 2 * WP + mm);
                a0 += w0.x * rv.x;
                a1 += w1.x * rv.x;
                a2 += w2.x * rv.x;
                a0 += w0.y * rv.y;
                a1 += w1.y * rv.y;
                a2 += w2.y * rv.y;
                if constexpr (NV == 4) {
                    a0 += w0.z * rv.z;
                    a1 += w1.z * rv.z;
                    a2 += w2.z * rv.z;
                    a0 += w0.w * rv.w;
                    a1 += w1.w * rv.w;
                    a2 += w2.w * rv.w;
                }
            }
        }
        static_assert(TBL >= 16, "runs are combined by 16- and 32-lane swaps");
#pragma unroll
        for (int o = TBL; o < 64; o <<= 1) {
            a0 = pair_sum(a0, o);
            a1 = pair_sum(a1, o);
            a2 = pair_sum(a2, o);
        }
        if (on && run == 0) {
            acc[p0] += a0;
            acc[p0 + 1] += a1;
            acc[p0 + 2] += a2;
        }
        __syncthreads();
    }

    // write column COL; reduce its batch when COL completes it
    template <int COL> STK_HD void put(T v) {
        cols[(COL % TBL) * PITCH + lane] = v;
        if constexpr (COL % TBL == TBL - 1)
            reduce(TBL, COL / TBL);
        else if constexpr (COL == NCOL - 1)
            reduce(NCOL % TBL, COL / TBL);
    }

    template <int Q, int N> STK_HD void coef(T bq) {
        if constexpr (N <= P + 1) {
            constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = N - K1 - K2;
            put<lam_gcol(P, K1, K2, K3)>(bq);
        }
    }

    template <int N, int J> STK_HD void layer_done(const T (&)[nidx(P + 2)]) {}

    // after order N: the E columns zh^k of order N - 1
    template <int N> STK_HD void order_done(const T (&b)[nidx(P + 2)]) {
        if constexpr (N >= 1) ecol<N, N - 1, 0>(b);
    }

    // zh^k = sum_i w_i (k_i+1) bt^{k+e_i} for every k of order M, in graded-lex order
    template <int N, int M, int A> STK_HD void ecol(const T (&b)[nidx(P + 2)]) {
        if constexpr (A < (M + 1) * (M + 2) / 2) {
            constexpr int Q = (M > 0 ? nidx(M - 1) : 0) + A;
            constexpr int K1 = kof1c(Q), K2 = kof2c(Q), K3 = M - K1 - K2;
            const T z = wl[0] * (T(K1 + 1) * b[gidx(K1 + 1, K2, K3)]) + wl[1] * (T(K2 + 1) * b[gidx(K1, K2 + 1, K3)]) +
                        wl[2] * (T(K3 + 1) * b[gidx(K1, K2, K3 + 1)]);
            put<lam_ebase(P, N) + A>(z);
            ecol<N, M, A + 1>(b);
        }
    }
};

template <int P, typename T> __global__ __launch_bounds__(64) void k_far_lambda(LambdaArgs a) {
    constexpr int NG = nidx(P + 1);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *acc = reinterpret_cast<T *>(lds_raw);
    T *cols = acc + 6 * NG;
    T *cw = cols + lam_tbl<T>() * lam_pitch<T>();
    T *dw = cw + 3 * lam_wp<T>();
    const int lane = threadIdx.x;
    const int32_t it = blockIdx.x;
    if (it >= a.nitems) return;
    const int32_t c = a.item_node[it];
    for (int q = lane; q < 6 * NG; q += 64) acc[q] = T(0);
    const double c0 = a.center[3 * c], c1 = a.center[3 * c + 1], c2 = a.center[3 * c + 2];
    const double rho = a.rho[c];
    const int32_t i1 = a.item_i1[it];
    for (int32_t i0 = a.item_i0[it]; i0 < i1; i0 += 64) {
        const bool in = i0 + lane < i1;
        const int64_t t = in ? a.inc_tgt[i0 + lane] : 0;
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
            cw[lam_wp<T>() * i + lam_wid<T>(lane)] = wl[i] * ri;
            dw[lam_wp<T>() * i + lam_wid<T>(lane)] = in ? dh[i] : T(0);
        }
        LambdaVisit<P, T> v{cols, cw, dw, acc, a.cpos, a.ckind, {wl[0], wl[1], wl[2]}, lane};
        T b[nidx(P + 2)];
        Coefs<P + 2, T, LambdaVisit<P, T>>::run(b, dh, tt, v);
    }
    __syncthreads();
    double *out = a.lambda + size_t(c) * 6 * NG;
    for (int q = lane; q < 6 * NG; q += 64) atomicAdd(out + q, double(acc[q]));
}

template <int P, typename T> struct TgradVisit {
    const T *W;   // cluster stream
    T dh[3], wl[3];
    T a1[3], a2[3], a3[3];
    T lag;        // the sums as they stood one layer back
    T zb[2][P + 3];  // zh of the two newest layers of the order below, by layer parity and k_1

    template <int Q, int N> STK_HD void coef(T) {}
    template <int N> STK_HD void order_done(const T (&)[nidx(P + 3)]) {}

    // after layer k3 = J of order N (layers 0..J of order N exist):
    //  term 1 for q of order N-1 in layer J-1 (<= P+1): (w.Ghat^q) (q_s+1) bt^{q+e_s}
    //  term 3 for k of order N-1 in layer J-1 (<= P+1): Ehat_s^k zh^k
    //  term 2 for k of order N-2 in layer J-2 (<= P+1):
    //      (dh.Ehat^k) sum_i w_i (k_i+1)(k_s+1+delta_is) bt^{k+e_i+e_s}
    //    = (dh.Ehat^k) (k_s+1) zh^{k+e_s}   ((k_i+1)(k_s+1+delta_is) = (k_s+1)(m_i+1) with
    //      m = k + e_s), so it reads the zh of layers J-2 and J-1 of order N-1, which the
    //      term-3 walk has just formed (for order P+2 they are formed for this use alone)
    // so each layer of order N is last read one layer later
    template <int N, int J> STK_HD void layer_done(const T (&b)[nidx(P + 3)]) {
        // the fence pins this layer's scalar loads after the sums of two layers back, so they
        // can be in flight while the previous layer is consumed
        const T *__restrict__ Wf = W + FarEval<P, T>::fence(lag);
        lag = a1[0] + a2[0] + a3[0];
        if constexpr (J >= 1 && N - 1 <= P + 1) walk13<N - 1, J - 1, N - J>(b, Wf);
        if constexpr (J >= 1 && N - 1 == P + 2) walkz<N - 1, J - 1, N - J>(b);
        if constexpr (J >= 2 && N - 2 <= P + 1) walk2<N - 2, J - 2, N - J>(Wf);
    }

    // zh^k = sum_i w_i (k_i+1) bt^{k+e_i}, kept for term 2
    template <int M, int K3, int K1> STK_HD T zh(const T (&b)[nidx(P + 3)]) {
        constexpr int K2 = M - K3 - K1;
        const T z = wl[0] * (T(K1 + 1) * b[gidx(K1 + 1, K2, K3)]) + wl[1] * (T(K2 + 1) * b[gidx(K1, K2 + 1, K3)]) +
                    wl[2] * (T(K3 + 1) * b[gidx(K1, K2, K3 + 1)]);
        zb[K3 & 1][K1] = z;
        return z;
    }

    template <int M, int K3, int K1> STK_HD void walkz(const T (&b)[nidx(P + 3)]) {
        (void)zh<M, K3, K1>(b);
        if constexpr (K1 > 0) walkz<M, K3, K1 - 1>(b);
    }

    // k of order M in layer k3 = K3, k1 = K1 .. 0
    template <int M, int K3, int K1> STK_HD void walk13(const T (&b)[nidx(P + 3)], const T *__restrict__ W) {
        constexpr int K2 = M - K3 - K1;
        constexpr int kk[3] = {K1, K2, K3};
        int pg = 0, pe = 0;
        stream_pos_c(kk, pg, pe);
        const T g = wl[0] * W[pg] + wl[1] * W[pg + 1] + wl[2] * W[pg + 2];
        const T bx = b[gidx(K1 + 1, K2, K3)], by = b[gidx(K1, K2 + 1, K3)], bz = b[gidx(K1, K2, K3 + 1)];
        a1[0] += g * (T(K1 + 1) * bx);
        a1[1] += g * (T(K2 + 1) * by);
        a1[2] += g * (T(K3 + 1) * bz);
        const T z = zh<M, K3, K1>(b);
        a3[0] += W[pe] * z;
        a3[1] += W[pe + 1] * z;
        a3[2] += W[pe + 2] * z;
        if constexpr (K1 > 0) walk13<M, K3, K1 - 1>(b, W);
    }

    template <int M, int K3, int K1> STK_HD void walk2(const T *__restrict__ W) {
        constexpr int K2 = M - K3 - K1;
        constexpr int kk[3] = {K1, K2, K3};
        int pg = 0, pe = 0;
        stream_pos_c(kk, pg, pe);
        const T sig = dh[0] * W[pe] + dh[1] * W[pe + 1] + dh[2] * W[pe + 2];
        // h_s = (k_s+1) zh^{k+e_s}: k+e_1 and k+e_2 lie in layer K3 of order M+1, k+e_3 in
        // layer K3+1
        a2[0] += sig * (T(K1 + 1) * zb[K3 & 1][K1 + 1]);
        a2[1] += sig * (T(K2 + 1) * zb[K3 & 1][K1]);
        a2[2] += sig * (T(K3 + 1) * zb[(K3 + 1) & 1][K1]);
        if constexpr (K1 > 0) walk2<M, K3, K1 - 1>(W);
    }

    STK_HD static constexpr void stream_pos_c(const int (&k)[3], int &g, int &e) {
        const int n = k[0] + k[1] + k[2], j = k[2], i = (n - j) - k[0];
        g = n == 0 ? 0 : stream_off(P, n, j) + 3 * i;
        e = stream_off(P, n + 1, j + 1) + stream_gpart(P, n + 1, j + 1) + 3 * i;
    }
};

// one wave per work item: a cluster and up to 64 of its incidences; each lane forms its
// target's term of this interaction and writes it to the incidence's slot
template <int P, typename T> __global__ __launch_bounds__(64, sizeof(T) == 4 ? 4 : 2) void k_far_tgrad(TgradArgs a) {
    constexpr int NG = nidx(P + 1);
    const int32_t it = xcd_group(a.nitems);
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int32_t c = __builtin_amdgcn_readfirstlane(a.item_node[it]);
    const int32_t i0 = a.item_i0[it];
    if (lane >= a.item_i1[it] - i0) return;
    const int64_t t = a.inc_tgt[i0 + lane];
    const int32_t slot = a.inc_slot[i0 + lane];
    const double d0 = a.tpos[3 * t] - a.center[3 * c], d1 = a.tpos[3 * t + 1] - a.center[3 * c + 1],
                 d2 = a.tpos[3 * t + 2] - a.center[3 * c + 2];
    const double rinv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double rho = a.rho[c];
    TgradVisit<P, T> v{static_cast<const T *>(a.wblk) + size_t(c) * 6 * NG,
                       {T(d0 * rinv), T(d1 * rinv), T(d2 * rinv)},
                       {T(a.ws[3 * t]), T(a.ws[3 * t + 1]), T(a.ws[3 * t + 2])},
                       {T(0), T(0), T(0)},
                       {T(0), T(0), T(0)},
                       {T(0), T(0), T(0)},
                       T(0)};
    T b[nidx(P + 3)];
    Coefs<P + 3, T, TgradVisit<P, T>>::run(b, v.dh, T(rho * rinv), v);
    const T f1 = T(-rinv / rho), f2 = T(-1.0 / rho), f3 = T(rinv);
    T *o = static_cast<T *>(a.part) + 3 * int64_t(slot);
    for (int s = 0; s < 3; ++s) o[s] = f1 * v.a1[s] + f2 * v.a2[s] + f3 * v.a3[s];
}

template <int P, typename T> void launch_far_lambda(const LambdaArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    hipLaunchKernelGGL((k_far_lambda<P, T>), dim3(a.nitems), dim3(64), (lam_lds_bytes<P, T>()), s, a);
    STK_CHECK_LAUNCH();
}

template <int P, typename T> void launch_far_tgrad(const TgradArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    hipLaunchKernelGGL((k_far_tgrad<P, T>), dim3(xcd_blocks(a.nitems)), dim3(64), 0, s, a);
    STK_CHECK_LAUNCH();
}

// ---- far source gradients from the moment adjoints ---------------------------------------
template <int P> struct SrcGrad {
    static constexpr int NM = nidx(P);
    // accumulate over every k of order <= P (compile-time walk in graded-lex order)
    template <int A>
    STK_HD static void walk(const double (&px)[P + 1], const double (&py)[P + 1], const double (&pz)[P + 1],
                            const double *__restrict__ L, const double f[3], const double hn[9], const double nu[3],
                            double gf[3], double gh[3], double gy[3]) {
        if constexpr (A < NM) {
            constexpr int K1 = kof1c(A), K2 = kof2c(A), K3 = ordc(A) - K1 - K2;
            const double *La = L + A * 12;
            const double mono = px[K1] * py[K2] * pz[K3];
            double pf = 0.0;
            for (int j = 0; j < 3; ++j) {
                gf[j] += mono * La[j];
                const double hl = nu[0] * La[3 + 3 * j] + nu[1] * La[4 + 3 * j] + nu[2] * La[5 + 3 * j];
                gh[j] += mono * hl;
                pf += f[j] * La[j];
            }
            for (int q = 0; q < 9; ++q) pf += hn[q] * La[3 + q];
            if constexpr (K1 > 0) gy[0] += double(K1) * (px[K1 - 1] * py[K2] * pz[K3]) * pf;
            if constexpr (K2 > 0) gy[1] += double(K2) * (px[K1] * py[K2 - 1] * pz[K3]) * pf;
            if constexpr (K3 > 0) gy[2] += double(K3) * (px[K1] * py[K2] * pz[K3 - 1]) * pf;
            walk<A + 1>(px, py, pz, L, f, hn, nu, gf, gh, gy);
        }
    }
};


__device__ inline int32_t node_of_item(const int32_t *__restrict__ off, int32_t nn, int32_t ch) {
    int32_t lo = 0, hi = nn;
    while (hi - lo > 1) {
        const int32_t m = (lo + hi) >> 1;
        if (off[m] <= ch)
            lo = m;
        else
            hi = m;
    }
    return lo;
}

template <int P> __global__ __launch_bounds__(256) void k_src_grad(SrcGradArgs a) {
    const int32_t ch = blockIdx.x;
    const int32_t node = node_of_item(a.coff, a.nn, ch);
    const int32_t first = a.start[node] + (ch - a.coff[node]) * CHUNK;
    const int32_t last = min(a.start[node] + a.count[node], first + CHUNK);
    const double *L = a.lm + size_t(node) * nidx(P) * 12;
    const int lev = a.level[node];
    for (int32_t j = first + threadIdx.x; j < last; j += 256) {
        double px[P + 1], py[P + 1], pz[P + 1];
        const double dx = a.pos[3 * int64_t(j)] - a.center[3 * node];
        const double dy = a.pos[3 * int64_t(j) + 1] - a.center[3 * node + 1];
        const double dz = a.pos[3 * int64_t(j) + 2] - a.center[3 * node + 2];
        px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
        for (int e = 1; e <= P; ++e) {
            px[e] = px[e - 1] * dx;
            py[e] = py[e - 1] * dy;
            pz[e] = pz[e - 1] * dz;
        }
        const double *wr = a.w12 + 12 * int64_t(j);
        const double f[3] = {wr[0], wr[1], wr[2]};
        double hn[9];
        for (int q = 0; q < 9; ++q) hn[q] = wr[3 + q];
        const double nu[3] = {a.geo[6 * int64_t(j) + 3], a.geo[6 * int64_t(j) + 4], a.geo[6 * int64_t(j) + 5]};
        double gf[3] = {0, 0, 0}, gh[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
        SrcGrad<P>::template walk<0>(px, py, pz, L, f, hn, nu, gf, gh, gy);
        double *o = a.part + (size_t(lev) * a.n + j) * 9;
        for (int q = 0; q < 3; ++q) {
            o[q] = gf[q];
            o[3 + q] = gh[q];
            o[6 + q] = gy[q];
        }
    }
}

template <int P> void launch_src_grad(const SrcGradArgs &a, int32_t nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_src_grad<P>), dim3(nitems), dim3(256), 0, s, a);
    STK_CHECK_LAUNCH();
}


}  // namespace stk
