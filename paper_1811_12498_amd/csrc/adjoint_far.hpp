// Far-field adjoint kernels (the transpose of the frozen-plan treecode operator).
//
// For L = sum_m w^m . u^m with the interaction lists, cluster centres and scales held
// fixed, one far interaction contributes (stk_math.hpp notation, scaled quantities)
//     L_mC = sum_q (w . Ghat^q) bt^q / R + sum_k (dh . Ehat^k) zh^k,
//     zh^k = sum_i w_i (k_i + 1) bt^{k + e_i},
// which is linear in the cluster stream (Ghat, Ehat).  Two kernels use it:
//   k_far_lambda  accumulates dL/dGhat_i^q = sum_m (w_i / R) bt^q and
//                 dL/dEhat_l^k = sum_m dh_l zh^k over the targets that accept the cluster
//                 (work items: runs of a cluster's incidences, 64 per pass whatever
//                 groups they come from; per order the wave writes its targets'
//                 coefficients to LDS and each lane sums whole columns);
//   k_far_tgrad   dL/dx for each target (one incidence per lane, the partial written to
//                 the incidence's slot in the target's list and the slots added in list
//                 order afterwards), from d/dx_s b^q = -(q_s + 1) b^{q + e_s}:
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
// k_far_lambda
// ---------------------------------------------------------------------------------
struct LambdaArgs {
    const double *tpos;        // sorted targets
    const double *ws;          // sorted adjoint seed w (m,3)
    int64_t m;
    const int32_t *item_node;  // work item -> cluster
    const int32_t *item_i0;    // work item -> its incidences [i0, i1) in the cluster-major view
    const int32_t *item_i1;
    const int32_t *inc_tgt;    // incidence -> sorted target
    const double *center, *rho;
    const int32_t *cpos;       // (columns): stream position of each LDS column
    const int32_t *ckind;      // (columns): 0 = G column (weights w / R), 1 = E column (weights dh)
    double *lambda;            // (nn, 6 nG) adjoint of the cluster streams, accumulated
    int32_t nitems;
};


// The LDS columns of k_far_lambda (one value per target lane) in the order they are
// formed: the G column of order 0, then per order n = 1 .. p + 2 the G columns of order n
// (n <= p + 1; layer k3 = 0 .. n, k2 = 0 .. n - k3 within a layer) followed by the E
// columns of order n - 1 (graded-lex order).  Every lam_tbl<T> consecutive columns form
// a batch, reduced over the 64 targets as soon as its last column is written, with
// 64 / lam_tbl<T> lanes per column each summing lam_tbl<T> targets (narrower batches in
// FP64 keep the LDS of a block small enough for more blocks per CU).
template <typename T> __host__ __device__ constexpr int lam_tbl() { return sizeof(T) == 8 ? 16 : 32; }
constexpr int LAM_TBL_MAX = 32;  // host column tables are padded to whole batches of this
// values per 16-byte LDS read
template <typename T> __host__ __device__ constexpr int lam_nv() { return 16 / int(sizeof(T)); }
// column row pitch (targets): 16-byte aligned rows whose 16-byte reads by consecutive
// columns fall in distinct banks
template <typename T> __host__ __device__ constexpr int lam_pitch() { return 64 + lam_nv<T>(); }
// weight table pitch and position: 16 pad bytes after each run of lam_tbl targets, so that
// every run starts 16-byte aligned and the runs read at once fall in distinct banks
template <typename T> __host__ __device__ constexpr int lam_wp() { return 64 + (64 / lam_tbl<T>()) * lam_nv<T>(); }
template <typename T> __host__ __device__ constexpr int lam_wid(int t) { return t + (t / lam_tbl<T>()) * lam_nv<T>(); }
__host__ __device__ constexpr int lam_ncol(int p) { return 2 * nidx(p + 1); }
// first column of the G columns of order n (n >= 0; past the last one for n > p + 1)
__host__ __device__ constexpr int lam_gbase(int p, int n) {
    if (n == 0) return 0;
    int c = 1;
    for (int m = 1; m < n; ++m) c += (m <= p + 1 ? (m + 1) * (m + 2) / 2 : 0) + m * (m + 1) / 2;
    return c;
}
// first column of the E columns of order n - 1 (n >= 1)
__host__ __device__ constexpr int lam_ebase(int p, int n) {
    return lam_gbase(p, n) + (n <= p + 1 ? (n + 1) * (n + 2) / 2 : 0);
}
// column of G^k, ||k|| = n <= p + 1
__host__ __device__ constexpr int lam_gcol(int p, int k1, int k2, int k3) {
    const int n = k1 + k2 + k3;
    int c = lam_gbase(p, n) + k2;
    for (int j = 0; j < k3; ++j) c += n - j + 1;
    return c;
}
// LDS of one work item: the stream accumulator (evaluation precision), one batch of
// columns and the two weight tables
template <int P, typename T> __host__ __device__ constexpr size_t lam_lds_bytes() {
    return sizeof(T) * (6 * size_t(nidx(P + 1)) + size_t(lam_tbl<T>()) * lam_pitch<T>() + 6 * size_t(lam_wp<T>()));
}

// ---------------------------------------------------------------------------------
// k_far_tgrad
// ---------------------------------------------------------------------------------
struct TgradArgs {
    const double *tpos, *ws;
    const int32_t *item_node, *item_i0, *item_i1;  // work items of up to 64 incidences of one cluster
    const int32_t *inc_tgt, *inc_slot;             // incidence -> sorted target, slot in its list
    const double *center, *rho;
    const void *wblk;
    void *part;   // (incidences, 3) T: each incidence's term, at its slot
    int32_t nitems;
};

// per source, from the moment adjoints of its node: dL/df, dL/dh, dL/dy (one partial
// per tree level)
struct SrcGradArgs {
    const double *pos, *geo, *w12, *center, *lm;
    const int32_t *start, *count, *coff, *level;
    int32_t nn;
    int64_t n;
    double *part;  // (nlevels, n, 9)
};

// defined in adjoint_far_impl.hpp, instantiated per Taylor order in adj_p*.hip / adjt_p*.hip
template <int P, typename T> void launch_far_lambda(const LambdaArgs &a, hipStream_t s);
template <int P, typename T> void launch_far_tgrad(const TgradArgs &a, hipStream_t s);
template <int P> void launch_src_grad(const SrcGradArgs &a, int32_t nitems, hipStream_t s);

}  // namespace stk
