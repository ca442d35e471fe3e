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

// ---------------------------------------------------------------------------------
// k_far_tgrad
// ---------------------------------------------------------------------------------
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
