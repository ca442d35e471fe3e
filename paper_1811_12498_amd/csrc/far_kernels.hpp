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
    const void *wblk;        // (nn, K, 6 nG) in T: each cluster's G/E stream per right-hand side
    const double *unear;     // (m,K,3) sorted near-field velocity
    const int32_t *tperm;    // sorted -> caller index
    double *u_out;           // (K,m,3) caller order
    int32_t ngroups;
    int32_t K;               // right-hand sides (a multiple of the kernel's block KB)
    int32_t sparse_max;      // entries with at most this many targets are done elsewhere (0: none)
    int32_t nsplit;          // parts of each group's far list, one wave each (grid z); 1: the
                             // wave adds the near part and writes u_out itself
    double *fpart;           // nsplit > 1: (nsplit, K, m, 3) each part's sums, sorted targets
};

// cluster-major items of the sparse far entries (one right-hand side)
struct FarSparseArgs {
    const double *tpos;
    const int32_t *item_node, *item_i0, *item_i1;
    const int32_t *inc_tgt, *inc_slot;
    const double *center, *rho;
    const void *wblk;
    void *part;              // (incidences, K, 3) T
    int32_t nitems;
    int32_t K;               // right-hand sides
};

// block index -> group: XCD x = blockIdx % 8 gets groups [x * per, (x + 1) * per)
__device__ inline int32_t xcd_group(int32_t ngroups) {
    const int32_t per = (ngroups + 7) >> 3;
    return int32_t(blockIdx.x & 7) * per + int32_t(blockIdx.x >> 3);
}
inline unsigned xcd_blocks(int32_t ngroups) { return unsigned(((ngroups + 7) >> 3) << 3); }

// block index -> work item for item lists whose cost varies along the list (one leaf or
// cluster per run of items, runs of very different lengths and leaf sizes): runs of
// CHUNK consecutive items are dealt to the eight XCDs in turn, so every XCD gets an even
// share of the work (contiguous eighths of the 1M-sphere near items differ by up to 1.5x
// in cost) while neighbouring items, which read the same source records or cluster
// streams, still share an L2.  The near-field items use runs of 16; the far field's
// cluster-major items, whose per-cluster streams are larger (FP64 in particular), runs of
// 256.  Indices run over [0, xcd_item_blocks(n)); those >= n have no item.
constexpr int32_t XCD_CHUNK_NEAR = 16, XCD_CHUNK_FAR = 256;
template <int32_t CHUNK> __device__ inline int32_t xcd_item() {
    const int32_t j = int32_t(blockIdx.x >> 3);
    return ((j / CHUNK) * 8 + int32_t(blockIdx.x & 7)) * CHUNK + j % CHUNK;
}
template <int32_t CHUNK> inline unsigned xcd_item_blocks(int32_t nitems) {
    const int32_t chunks = (nitems + CHUNK - 1) / CHUNK;
    return unsigned(((chunks + 7) / 8) * 8 * CHUNK);
}

// defined in far_impl.hpp, instantiated per Taylor order in far_p*.hip / fark_p*.hip
template <int P, typename T, int KB> void launch_far(const FarArgs &a, hipStream_t s);
template <int P, typename T, int KB> void launch_far_sparse(const FarSparseArgs &a, hipStream_t s);

}  // namespace stk
