// Internal declarations shared by the HIP translation units of libstokestree.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "stokestree.h"

namespace stk {

// ---------------------------------------------------------------------------------
// errors: internal code throws stk::Error; the C-ABI layer converts it to a status
// ---------------------------------------------------------------------------------
struct Error : std::runtime_error {
    stk_status status;
    Error(stk_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define STK_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            throw ::stk::Error(e_ == hipErrorOutOfMemory ? STK_ENOMEM : STK_EDEVICE,               \
                               std::string(#call) + ": " + hipGetErrorString(e_));                 \
        }                                                                                          \
    } while (0)

#define STK_CHECK_LAUNCH() STK_HIP(hipGetLastError())

inline void require(bool ok, const std::string &msg) {
    if (!ok) throw Error(STK_EINVAL, msg);
}

// ---------------------------------------------------------------------------------
// device buffer (grow-only, freed with its owner)
// ---------------------------------------------------------------------------------
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // Ensure capacity; contents are not preserved.
    void reserve(size_t b) {
        if (b <= bytes) return;
        release();
        size_t want = b < 256 ? 256 : b;
        STK_HIP(hipMalloc(&p, want));
        bytes = want;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------------
// small device-to-host reads: the sizes the host needs before its next launch (list
// lengths, node and chunk counts).  One kernel copies up to PEEK_MAX 4- or 8-byte device
// values into pinned host slots, then one stream synchronisation (a pageable copy would
// cost a round trip of its own per value).
// ---------------------------------------------------------------------------------
constexpr int PEEK_MAX = 32;
struct HostPeek {
    int64_t *h = nullptr;  // pinned, PEEK_MAX slots (allocated on first use, kept with the owner)
    int64_t *d = nullptr;  // the same slots as the device sees them
    HostPeek() = default;
    HostPeek(const HostPeek &) = delete;
    HostPeek &operator=(const HostPeek &) = delete;
    ~HostPeek() {
        if (h) (void)hipHostFree(h);
    }
};
struct PeekSrc {
    const void *p;  // device address
    int bytes;      // 4: int32 (sign-extended); 8: int64 or double (raw bits)
};
// Enqueue the copy of src[0..n) (1 <= n <= PEEK_MAX) on s, synchronise s, and return the
// values in out[0..n).  peek_start only enqueues the copy (peek_wait completes it).
void peek(HostPeek &pk, hipStream_t s, int n, const PeekSrc *src, int64_t *out);
void peek_start(HostPeek &pk, hipStream_t s, int n, const PeekSrc *src);
// The slots as the device sees them (allocated if needed), for a kernel that writes its
// results there itself; peek_wait then synchronises s and returns slots [0, n).
int64_t *peek_slots(HostPeek &pk);
void peek_wait(HostPeek &pk, hipStream_t s, int n, int64_t *out);

template <class T> inline T *reserve(DBuf &b, size_t n) {
    b.reserve(n * sizeof(T));
    return b.as<T>();
}

// ---------------------------------------------------------------------------------
// tree handle
// ---------------------------------------------------------------------------------
// One record per node for the MAC traversal: everything a visit reads, in one 64-byte line.
struct alignas(64) TravNode {
    double c[3];  // centre
    double r;     // radius
    int32_t nchild, child0, count, pad[5];
};

struct Tree {
    int device = 0;
    int64_t n = 0;
    int32_t n0 = 0;
    double lo[3] = {0, 0, 0}, L = 0.0, scale = 0.0;
    bool degenerate = false;
    int32_t nnodes = 0, nlevels = 0;
    std::vector<int32_t> level_begin;  // host: first node of each level (+ end sentinel)

    // sources in Morton order
    DBuf keys, perm;            // uint64 keys, int32 sorted->input
    DBuf pos;                   // double (n,3) sorted positions, row-major
    // node table (SoA)
    DBuf nlevel, nparent, nchild0, nnchild, nstart, ncount;   // int32
    DBuf nbmin, nbmax, ncenter;  // double (nn,3)
    DBuf nradius, nrho;          // double (nn)
    DBuf trav;                   // TravNode (nn): the fields above that the traversal reads
    // work chunks over (node, particle range) for per-node reductions
    DBuf chunk_off;              // int32 (nn + 1): first chunk of each node
    int32_t nchunks = 0;
    DBuf leaf_coff;              // int32 (nn + 1): the same over leaves only (0 chunks for inner nodes)
    int32_t nleafchunks = 0;

    // moments state
    bool have_moments = false;
    int32_t p = -1, k_rhs = 0;
    stk_precision prec = STK_FP64;
    DBuf mom;     // double (nn, nm, 12*K): channels 0..2 = M_j, 3..11 = Mt_jl (3 + 3j + l)
    DBuf mom_up;  // double, as mom: each node's moments moved to its parent's centre
    DBuf mom_part;  // double: the leaves' chunk partials (moments may run beside an evaluation)
    DBuf wblk;    // T (nn, nb, 12*K): scaled far-field channel blocks
    DBuf wreg;    // double (nn, reg_stream_len(p)): regularized far-field streams
    DBuf geo;     // double (n, 6): sorted (y, nu) per source
    DBuf wts;     // T (n, K, 6): sorted (f, h) per source and right-hand side
    DBuf w12;     // double (n, K, 12): sorted (f_j, h_j nu_l) for the moments

    // reusable scratch for evaluation
    DBuf s_keys, s_vals, s_keys2, s_vals2, s_hist, s_tmp;
    DBuf s_scan;                   // tile sums of scan_exclusive_i32
    DBuf s_slot;                   // per-group list slots of the one-pass traversal
    // their capacity: a quarter above the longest group lists of the last evaluation with
    // this tree (0: none yet)
    int32_t slot_far = 0, slot_near = 0;
    DBuf s_bm;                     // operand blocks of the matrix-core far field
    HostPeek peek;                 // host slots for the sizes read back during a build or evaluation
};

// lists re-sorted by node (cluster-major / leaf-major) and their work items
struct TransposedLists {
    DBuf ent, ent_off, ent_group, item_node, item_a, item_b;
    int32_t nitems = 0;
};

// ---------------------------------------------------------------------------------
// plan handle: a tree plus one target set's interaction lists
// ---------------------------------------------------------------------------------
// Cluster-major view of (a filtered subset of) group-major lists: every (target, node)
// incidence of the included entries placed in a node-sorted array, work items of up to 64
// incidences of one node, and per target the slots of its incidences in the order of its
// own list.
struct ClusterMajor {
    DBuf keys, ent;                // uint64 / int32 (entries): entries sorted by node
    DBuf pc, pos;                  // int32: incidences of each sorted entry; sorted position of each entry
    DBuf incoff;                   // int32 (entries + 1): first incidence of each sorted entry
    DBuf eoff, loff;               // int32 (nn + 1): first sorted entry / first incidence of each node
    DBuf icnt, ioff;               // int32: items per node (nn), their offsets (nn + 1)
    DBuf tcnt, toff;               // int32: included entries per target (m), first slot (m + 1)
    DBuf inc_tgt, inc_slot;        // int32 (incidences): sorted target and slot of each incidence
    DBuf item_node, item_i0, item_i1;  // int32 (items)
    DBuf part;                     // T (incidences, K, 3): per-incidence partial velocities
    int64_t n_inc = 0;
    int32_t n_items = 0;
    // the build's own sort and scan scratch and readback slots, so that two views can be
    // built at once on two streams; nk = entries in the sorted array
    DBuf s_keys2, s_vals2, s_hist, s_scan;
    HostPeek peek;
    int64_t nk = 0;
    bool nk_pending = false;
};

// scratch of the adjoint, kept with the plan for repeated backward calls
struct AdjScratch {
    DBuf ws, gt_near, gt_far, lambda, lm, part, gs;
    TransposedLists far_t, near_t;  // far_t: the cluster-adjoint work items
    ClusterMajor far_cm;            // every far entry, cluster major
};

// kernel variants of one evaluation (chosen per architecture, p, K and precision)
struct Tiles {
    int32_t far_kb = 1;      // right-hand sides per pass of the far-field kernel (1, 2, 4)
    int32_t near_kb = 1;     // right-hand sides per pass of the VALU near-field kernel
    bool near_mfma = false;  // near field on the matrix cores (FP32)
    bool far_mfma = false;   // far field on the matrix cores (FP32)
    int32_t far_cm = 0;      // FAR_CM_AUTO / FAR_CM_ON / FAR_CM_OFF
    int32_t far_split = 0;   // parts of each group's far list, a wave each (1..FAR_SPLIT_MAX; 0: automatic)
};

// far_cm modes: every far entry cluster major when the group lists' lanes are less than
// FAR_CM_UTIL full (auto), always (on), or never (off: only the split of sparse entries
// with one right-hand side)
constexpr int32_t FAR_CM_AUTO = 0, FAR_CM_ON = 1, FAR_CM_OFF = 2;
constexpr double FAR_CM_UTIL = 0.75;
// far_split: at most this many parts; the automatic choice is the smallest number of parts
// that gives at least FAR_SPLIT_ROUNDS waves per wave slot of four waves per SIMD
constexpr int32_t FAR_SPLIT_MAX = 4, FAR_SPLIT_ROUNDS = 12;
// cluster-major lists index incidences with int32
constexpr int64_t CM_MAX_INC = (int64_t(1) << 31) - 64;

struct Plan {
    Tree *tree = nullptr;
    bool owns_tree = false;
    int64_t m = 0;
    double theta = 0.0;
    int32_t ngroups = 0;
    DBuf tpos;                     // double (m,3) targets in Morton order
    DBuf tperm;                    // int32 sorted -> caller index
    // the targets in use: tpos / tperm, or the tree's sorted sources and their permutation
    // when the targets are the sources
    const double *tpos_p = nullptr;
    const int32_t *tperm_p = nullptr;
    DBuf far_off, near_off;        // int32 (ngroups + 1)
    DBuf far_node, near_node;      // int32 entries
    DBuf far_mask, near_mask;      // uint64 entries (lane masks of the 64-target group)
    DBuf cnt_far, cnt_near, cnt_pairs;  // int32 per sorted target
    DBuf far_inc;                       // int64 (4): far (target, cluster) and near (target, leaf) pairs, longest far and near group lists
    int64_t n_far_entries = 0, n_near_entries = 0, n_far_inc = 0;
    // cluster-major views of the group lists: the near field (every near entry) and, for
    // one right-hand side, the far entries that apply to few targets of their group
    ClusterMajor ncm, fcm;
    int32_t far_sparse_max = 0;       // threshold of the last evaluation's sparse far split
    Tiles tiles;                      // kernel variants used by the last evaluation
    bool forced = false;              // use `force` instead of the table (autotuning)
    // if set, computed on another stream: the evaluation's stream waits on records_ready
    // before the near field (which reads the source records) and on moments_ready before
    // the far field (which reads the clusters' streams)
    hipEvent_t records_ready = nullptr, moments_ready = nullptr;
    // if set, a stream on which the evaluation builds the sparse far entries' view while
    // its own stream builds the near field's; ev: the events that order the two
    hipStream_t aux = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    double reg_eps = -1.0;            // >= 0: the last evaluation used the regularized kernels with this eps
    Tiles force;
    AdjScratch adj;
    DBuf far_part;                    // double (parts, K, m, 3): sums of the split group-major far field

    ~Plan();
};

// ---------------------------------------------------------------------------------
// launch helpers implemented in the .hip files
// ---------------------------------------------------------------------------------
constexpr int GROUP = 64;  // targets per wavefront group
constexpr int CHUNK = 512;   // particles per reduction work item

// radix sort of (uint64 key, int32 value) pairs; sorts keys[0..n) in place using
// scratch buffers owned by `t`.  Stable.  `bits` = number of low key bits to sort.
void radix_sort_pairs(Tree &t, uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);
// the same with explicit scratch (keys2: n uint64, vals2: n int32, hist: the tile histograms)
void radix_sort_pairs(DBuf &keys2, DBuf &vals2, DBuf &hist, uint64_t *keys, int32_t *vals, int64_t n, int bits,
                      hipStream_t s);
// exclusive scan of int32 in[0..n) into out[0..n]; out[n] = total.  Long inputs use
// `scratch` for per-tile sums (in and out must not overlap).
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, DBuf &scratch, hipStream_t s);
// exclusive scans of a and b (length n) into oa and ob (oa[n], ob[n] = the totals), and
// stats = {sum of c, sum of d (int64), max of a, max of b}; one launch for n <= 65,536
void scan2_stats(const int32_t *a, int32_t *oa, const int32_t *b, int32_t *ob, const int32_t *c, const int32_t *d,
                 int64_t n, long long *stats, DBuf &scratch, hipStream_t s);

void build_tree(Tree &t, const double *src, int64_t n, int32_t n0, hipStream_t s);
// records_done, if given, is recorded on s once the per-source records (what the near
// field reads) are written, before the moments themselves
void compute_moments(Tree &t, const double *f, const double *h, const double *nu, int32_t k, int32_t p,
                     stk_precision prec, hipStream_t s, hipEvent_t records_done = nullptr);
// same_as_sources: the targets are exactly the tree's sources (same array), so their
// Morton order is the tree's and they are not sorted again
void evaluate(Tree &t, Plan &plan, const double *tgt, int64_t m, double theta, double *u_out, bool same_as_sources,
              hipStream_t s);
// the first part of evaluate: targets in Morton order and Algorithm 1's interaction lists
void build_lists(Tree &t, Plan &plan, const double *tgt, int64_t m, double theta, bool same_as_sources,
                 hipStream_t s);
// the same evaluation with the regularized Stokeslet and stresslet of parameter eps (FP64
// tree and moments, one right-hand side; regularized.hip)
void evaluate_regularized(Tree &t, Plan &plan, const double *tgt, int64_t m, double theta, double eps,
                          double *u_out, bool same_as_sources, hipStream_t s);
// gradients of L = sum_m w^m . u^m for the plan's frozen operator (any output may be
// NULL); w and the outputs in the caller's orders
void adjoint(Plan &plan, const double *w, double *grad_f, double *grad_h, double *grad_targets,
             double *grad_sources, hipStream_t s);
// kernel-variant table (tiles.hip)
Tiles default_tiles(int K, stk_precision prec);
bool tiles_valid(const Tiles &t, int K, stk_precision prec);
Tiles tiles_for(int p, int K, stk_precision prec);
bool tiles_lookup(int p, int K, stk_precision prec, Tiles *out);
void tiles_set(int p, int K, stk_precision prec, const Tiles *t);
void tiles_save(const char *path);
int tiles_load(const char *path);
Tiles autotune(int p, int K, stk_precision prec, int64_t n, double theta, int32_t n0, double *best_ms, hipStream_t s);

// Build cm from group-major lists (off: ngroups + 1 offsets, node/mask: ne entries), keeping
// the entries whose lane mask has at most max_pc bits (64: all).  tcount: per-target number
// of kept entries if known (sorted order), else NULL (counted here).  Synchronises s once
// or twice.  The build in three stages, each ending at (the request of) a host readback, so
// that a caller can interleave two builds on two streams: cm_stage1, cm_stage2, cm_stage3
// with the same arguments, in order.
struct CmInput {
    const int32_t *off, *node;
    const uint64_t *mask;
    int64_t ne;
    int32_t ng;
    int64_t m;
    int max_pc;
    const int32_t *tcount;
};
void cluster_major(Tree &t, ClusterMajor &cm, const int32_t *off, const int32_t *node, const uint64_t *mask,
                   int64_t ne, int32_t ng, int64_t m, int max_pc, const int32_t *tcount, hipStream_t s);
void cm_stage1(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s);
void cm_stage2(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s);
void cm_stage3(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s);
// near field of a plan whose group-major near lists are filled: unear (m,K,3), sorted
// target order, K = the tree's right-hand sides
// reduce = false leaves the per-target sums of the partials to a later pass (the partials
// stay in plan.ncm.part).  near_field = the leaf-major view (cluster_major of the near lists)
// then near_kernels.
void near_field(Tree &t, Plan &plan, double *unear, hipStream_t s, bool reduce = true);
void near_kernels(Tree &t, Plan &plan, double *unear, hipStream_t s, bool reduce);
// far entries with at most max_pc targets, cluster major: adds their velocities (every
// right-hand side) to unear (m,K,3); the group-major far kernel then skips entries of at
// most max_pc targets.  FAR_SPARSE_MAX is the split used by default with one right-hand
// side; max_pc = 64 takes every far entry.
constexpr int FAR_SPARSE_MAX = 32;
// add = false leaves the per-target sums to a later pass (the partials stay in plan.fcm.part).
// far_sparse_run: the kernels on a view plan.fcm already built.
void far_sparse(Tree &t, Plan &plan, double *unear, int max_pc, hipStream_t s, bool add = true);
void far_sparse_run(Tree &t, Plan &plan, double *unear, int max_pc, hipStream_t s, bool add);
// FP64 direct sum: k_direct sums `chunk` consecutive sources per wave for 64 targets into
// partial velocities (3 m nch doubles), k_direct_reduce adds them in chunk order; the shape
// depends only on (m, n)
struct DirectShape {
    int32_t chunk, nch;
};
DirectShape direct_shape(int64_t m, int64_t n);
void direct_launch(const double *tgt, int64_t m, const double *src, int64_t n, const double *f, const double *h,
                   const double *nu, const DirectShape &d, double *part, double *u, hipStream_t s);
void direct_sum(const double *tgt, int64_t m, const double *src, int64_t n, const double *f, const double *h,
                const double *nu, int32_t k, double *u_out, hipStream_t s);
// the same sum with the partials in a fixed per-device array (noalloc.hip): targets in
// slices of direct_noalloc_slice(m, n) (0 when 64 targets do not fit)
int64_t direct_noalloc_slice(int64_t m, int64_t n);
void direct_sum_noalloc(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                        const double *h, const double *nu, int32_t k, double *u_out, hipStream_t s);

// phase timing (profile.hip); phases are the STK_PHASE_* values of the public header
void prof_mark(int phase, hipStream_t s);
void prof_enable(bool on);
void prof_read(double *ms, int64_t *count);

inline int nm_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

}  // namespace stk
