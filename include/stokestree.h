/*
 * stokestree.h -- C-ABI of the MI355X (gfx950) treecode for 3D Stokeslets and
 * stresslets of Wang, Tlupova & Krasny, "A Treecode Algorithm for 3D Stokeslets
 * and Stresslets" (arXiv 1811.12498).
 *
 * The library evaluates, at targets x^m, the velocity of eq. StoStre (Sec. 1)
 *
 *     u_i(x^m) = sum_n S_ij(x^m, y^n) f_j^n + sum_n T_ijl(x^m, y^n) h_j^n nu_l^n
 *
 * with S and T exactly as printed in eqs. Stokeslet and stresslet (no 1/(8 pi)
 * prefactor, T positive, d = x - y target minus source).  A pair with x == y is
 * skipped (the n != m exclusion); targets may be disjoint from the sources.
 * Algorithm 1 (Sec. 5) is followed per target: an octree of source clusters,
 * the MAC r/R <= theta (eq. MAC), the order-p Cartesian Taylor far field
 * (eqs. S_final and T_final built on the Coulomb recurrence, recurrence_1) and
 * the contracted direct sum of Sec. 4.1 for leaves that fail the MAC.
 *
 * Conventions for every entry point:
 *   - Arrays named "device" are caller-owned device pointers (any allocation
 *     visible to the current HIP device), FP64, contiguous, row-major.  Arrays
 *     named "host" are caller-owned host memory.
 *   - (N,3) means N rows of (x, y, z); (K,N,3) means K consecutive (N,3) blocks,
 *     one per right-hand side.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = the default stream).
 *     Entry points that must size device buffers from data (tree build, list
 *     construction) synchronise that stream before returning; the others return
 *     after enqueueing.  Input arrays must stay valid until the stream has
 *     consumed them.
 *   - Handles (stk_tree, stk_plan) are owned by the library and released with
 *     the matching *_destroy call.  A handle is bound to the device that was
 *     current when it was created and must be used with that device current.
 *     Calls that use one handle must not overlap; distinct handles are
 *     independent.
 *   - Every entry point returns a stk_status.  Arguments are validated before
 *     any work is enqueued (STK_EINVAL); a failed HIP call yields STK_EDEVICE and
 *     an allocation failure STK_ENOMEM.  stk_last_error() returns a message for
 *     the last non-OK status of the calling thread.  No C++ exception crosses the
 *     ABI.  NaN/Inf inputs are not checked; they propagate.
 */
#ifndef STOKESTREE_H
#define STOKESTREE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stk_tree stk_tree; /* sources in Morton order, octree, moments  */
typedef struct stk_plan stk_plan; /* a tree plus one target set's interaction lists */

typedef enum {
    STK_OK = 0,
    STK_EINVAL = -1,  /* bad argument or parameter                               */
    STK_ENOMEM = -2,  /* device allocation failed                                 */
    STK_EDEVICE = -3, /* a HIP call failed                                        */
    STK_ESTATE = -4   /* call out of order (e.g. evaluate before compute_moments) */
} stk_status;

typedef enum {
    /* All arithmetic in FP64. */
    STK_FP64 = 0,
    /* Far and near fields in FP32 with compensated per-target accumulators and an
     * FP64 final sum; positions, normals and the pair quantities d = x - y and
     * d.nu are formed in FP64 (on a surface with nu the normal, d.nu = O(|d|^2),
     * so rounding them to FP32 would dominate the error); moments accumulate in
     * FP64 and are rounded once for the FP32 contraction. */
    STK_MIXED = 1
} stk_precision;

/* Largest Taylor order accepted (the paper uses p = 0..10). */
#define STK_P_MAX 10
/* Deepest octree level (21-bit integer coordinates per axis). */
#define STK_MAX_LEVEL 21

/* Build the octree of Sec. 5 over n source points.
 *   src  device (n,3) source positions y^n.
 *   n0   leaf capacity N0 >= 1: a node is split while it holds more than n0
 *        points and its level is below STK_MAX_LEVEL (so leaves hold <= n0
 *        points except at the deepest level).
 * The root cube is [lo, lo + L]^3 with lo the componentwise minimum and L the
 * largest extent; a point's integer coordinate per axis is
 * q = min(2^21 - 1, floor((y - lo) * (2^21 / L))) and children are visited in
 * Morton order (x bit most significant).  Each node's centre y_c is the centre of
 * the tight bounding box of its points and its radius r the largest |y - y_c|
 * (Sec. 2 and the box shrinking of Sec. 6).  If all points coincide (L = 0) the
 * tree is one leaf.  Synchronises `stream`.  *out receives the new handle. */
stk_status stk_build_tree(const double *src, int64_t n, int32_t n0, void *stream, stk_tree **out);

/* Compute the cluster moments of Sec. 2 for every node of `t`,
 *   M_j^k(C) = sum_{y^n in C} (y^n - y_c)^k f_j^n,
 *   Mt_jl^k(C) = sum_{y^n in C} (y^n - y_c)^k h_j^n nu_l^n,    ||k|| <= p,
 * for K = k_rhs right-hand sides, and the per-node blocks the far field reads.
 *   f, h  device (K,n,3) weights in the input order of the sources.
 *   nu    device (n,3) normals (used as given; normalising is the caller's job).
 *   p     Taylor order, 0 <= p <= STK_P_MAX.    prec  arithmetic of evaluation.
 * Moments are always accumulated in FP64.  Replaces any earlier moments. */
stk_status stk_compute_moments(stk_tree *t, const double *f, const double *h, const double *nu, int32_t k_rhs,
                               int32_t p, stk_precision prec, void *stream);

/* Evaluate the treecode velocity (Algorithm 1) at m targets with the moments of
 * the last stk_compute_moments on `t`.
 *   targets  device (m,3), m >= 1; may or may not coincide with the sources.
 *   theta    MAC parameter, 0 <= theta < 1: a node is used through its Taylor
 *            expansion iff R > 0 and r <= theta * R (R = |x - y_c|).
 *   u_out    device (K,m,3), overwritten (K = the k_rhs of the moments).  The K
 *            right-hand sides share the tree, the interaction lists and, for each
 *            target-cluster pair, the Taylor coefficients of recurrence_1.
 *   keep_plan  if non-NULL, receives a plan holding the targets' interaction
 *            lists (for stk_evaluate_adjoint and stk_plan_counts); it refers to
 *            `t`, which must outlive it.
 * Synchronises `stream` once (to size the interaction lists). */
stk_status stk_evaluate_tree(stk_tree *t, const double *targets, int64_t m, double theta, double *u_out,
                             stk_plan **keep_plan, void *stream);

/* One call: build the tree, compute moments and evaluate (eq. StoStre by
 * Algorithm 1).  Arguments as above; if keep_plan is non-NULL the plan owns the
 * tree it was built on.  The moments are computed on a second stream of the
 * library's (one per device, default priority, kept until the process ends) that
 * waits for `stream`'s work up to the tree and that `stream` waits for before the
 * near field, so f, h and nu follow the same rule as the other inputs and all work
 * of the call is ordered before what the caller enqueues on `stream` after it.
 * Concurrent calls from several host threads on one device share that stream:
 * their moments run one after another. */
stk_status stk_evaluate(const double *targets, int64_t m, const double *sources, int64_t n, const double *f,
                        const double *h, const double *nu, int32_t k_rhs, int32_t p, double theta, int32_t n0,
                        stk_precision prec, double *u_out, stk_plan **keep_plan, void *stream);

/* Adjoint of the treecode operator of `plan` (derived from eq. S_final, eq. T_final,
 * recurrence_1, the moments of Sec. 2 and the contracted pair of Sec. 4.1): for
 * L = sum_m w^m . u^m, the gradients with respect to the weights f and h, the source
 * positions and the target positions, with the plan's interaction lists, cluster
 * membership, centres, radii and scales held fixed (the discrete operator the forward
 * call applied).  The plan must come from a one-right-hand-side evaluation.
 *   w             device (m,3) in the caller's target order.
 *   grad_f, grad_h, grad_sources   device (n,3) in the caller's source order, or NULL.
 *   grad_targets  device (m,3) in the caller's target order, or NULL.
 * Outputs are overwritten.  Source-side sums over clusters use FP64 atomic additions,
 * so the last bits can differ between runs; everything else is deterministic.
 * Synchronises `stream` (to size the transposed lists).  Arithmetic follows the
 * plan's precision. */
stk_status stk_evaluate_adjoint(stk_plan *plan, const double *w, double *grad_f, double *grad_h,
                                double *grad_targets, double *grad_sources, void *stream);

/* The treecode with regularized Stokeslets and stresslets, the extension Sec. 7 names as
 * future work (kernels of the method of regularized Stokeslets, Cortez 2001 and
 * Cortez-Fauci-Medovikov 2005, normalised like eqs. Stokeslet and stresslet), FP64, one
 * right-hand side.  With R^2 = |x - y|^2 + epsilon^2 and d = x - y:
 *   u_i(x) = sum_n S^eps_ij f_j + T^eps_ijl h_j nu_l,
 *   S^eps_ij  = delta_ij (|d|^2 + 2 epsilon^2)/R^3 + d_i d_j/R^3,
 *   T^eps_ijl = [d_i d_j d_l + (epsilon^2/2)(delta_ij d_l + delta_jl d_i + delta_il d_j)]/R^5
 * (T^eps is -1/6 of the stress of the regularized Stokeslet's flow).  With epsilon > 0
 * every pair is finite and summed, the coincident one included (it adds 2 f/epsilon);
 * epsilon = 0 is eq. StoStre and skips it.  Same tree, moments, MAC (eq. MAC) and lists as
 * stk_evaluate (Algorithm 1); the far field is the order-p Taylor expansion of the
 * regularized kernels about each accepted cluster's centre (particle-cluster form of
 * Sec. 3 with coefficients from recurrence_1 generalised to R and to the exponents
 * -1, -3, -5).  Arguments and layouts as stk_evaluate with k_rhs = 1 (u_out (m,3) FP64,
 * caller's target order); epsilon finite and >= 0, else STK_EINVAL.  Synchronises
 * `stream` before returning. */
stk_status stk_evaluate_regularized(const double *targets, int64_t m, const double *sources, int64_t n,
                                    const double *f, const double *h, const double *nu, double epsilon, int32_t p,
                                    double theta, int32_t n0, double *u_out, void *stream);

/* Exact O(m n) direct sum of eq. StoStre in FP64 (contracted form of Sec. 4.1),
 * the reference the treecode is measured against.  Same array conventions. */
stk_status stk_direct(const double *targets, int64_t m, const double *sources, int64_t n, const double *f,
                      const double *h, const double *nu, int32_t k_rhs, double *u_out, void *stream);

/* For callers that cannot allocate device memory (work under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): stk_direct with the partial sums in
 * a fixed device array of STK_DIRECT_NOALLOC_SCRATCH_BYTES that each device holds until
 * the process ends, so the call allocates nothing (stk_direct allocates 24 m ceil(n/c)
 * bytes per call, c the source chunk of 512..8192).  Same arguments, conventions and
 * kernels, and results bit-identical to stk_direct's.  Targets are processed in slices
 * whose partial sums fit the array; fails with STK_EINVAL when 64 targets do not fit
 * (n above about 1.7e8 sources).  Every call on a device shares that device's array:
 * calls that overlap on one device (on different streams, or from several threads
 * without ordering) race and give wrong results.  The first call on a device looks up
 * the array's device address (hipGetSymbolAddress). */
#define STK_DIRECT_NOALLOC_SCRATCH_BYTES (32u << 20)
stk_status stk_direct_noalloc(const double *targets, int64_t m, const double *sources, int64_t n,
                              const double *f, const double *h, const double *nu, int32_t k_rhs, double *u_out,
                              void *stream);

/* Introspection, for verification and reporting. */
/* nnodes, number of levels, and root = (lo_x, lo_y, lo_z, L). Host outputs. */
stk_status stk_tree_info(const stk_tree *t, int64_t *nnodes, int32_t *nlevels, double root[4]);
/* Copy the node table to host arrays of length nnodes (3*nnodes for boxes and
 * centres) and perm (length n: sorted position -> input index).  Nodes are
 * numbered breadth first, each level in Morton order.  Any pointer may be NULL. */
stk_status stk_tree_export(const stk_tree *t, int32_t *perm, int32_t *level, int32_t *parent, int32_t *child0,
                           int32_t *nchild, int32_t *start, int32_t *count, double *bmin, double *bmax,
                           double *center, double *radius);
/* Copy right-hand side `rhs`'s FP64 moments to host arrays M (nnodes,nm,3) and
 * Mt (nnodes,nm,3,3), nm = (p+1)(p+2)(p+3)/6, k in graded-lex order
 * (n = 0..p; k1 = n..0; k2 = n-k1..0). */
stk_status stk_tree_export_moments(const stk_tree *t, int32_t rhs, double *M, double *Mt);
/* Per-target interaction counts of a plan, in the caller's target order (host
 * arrays of length m): far-field nodes, near-field leaves, near-field pairs. */
stk_status stk_plan_counts(const stk_plan *plan, int64_t *nfar, int64_t *nnear, int64_t *npairs);
/* Copy a plan's interaction lists (Alg. 1: the clusters accepted by eq. MAC, or the
 * leaves summed directly) to host arrays.  kind 0 = far field, 1 = near field.  Targets
 * are processed in groups of 64 consecutive Morton-sorted targets; group g's entries
 * are off[g] .. off[g+1]-1 (off has ngroups + 1 entries), entry e applies node[e]
 * (numbered as in stk_tree_export) to the targets whose lane bit is set in mask[e]:
 * bit l of mask[e] is sorted target 64 g + l, i.e. caller target tperm[64 g + l]
 * (tperm has m entries).  node and mask hold stk_plan_info's entry count for the kind.
 * Any pointer may be NULL.  EINVAL: kind not 0 or 1. */
stk_status stk_plan_export_lists(const stk_plan *plan, int32_t kind, int32_t *off, int32_t *node, uint64_t *mask,
                                 int32_t *tperm);

/* Kernel variants ("tiles") of the far and near fields, per (device architecture, p,
 * K = k_rhs, precision).  Not part of the paper's method: they change only how the
 * sums are scheduled on the GPU (and, for near_mfma, the FP32 summation order).
 *   far_kb     right-hand sides per pass of the far-field kernel: 1, 2 or 4, dividing K
 *              (FP64: 1).  Each pass shares one Taylor-coefficient recurrence.
 *   near_kb    right-hand sides per pass of the VALU near-field kernel: 1, 2 or 4,
 *              dividing K (FP64: 1).
 *   near_mfma  1: near field on the matrix cores (FP32 mixed precision only), 16
 *              right-hand sides per pass; near_kb is then unused.
 *   far_mfma   1: far field on the matrix cores (FP32 mixed precision only), 16
 *              right-hand sides per pass; far_kb is then unused.
 *   far_cm     0 (automatic): as 1 when the far group lists' lane masks are less than
 *              75% full on average, else as 2;  1: every far entry cluster major (64 of a
 *              cluster's targets per pass, whatever groups they belong to; each target's
 *              terms added in the order of its own list; not with far_mfma; EINVAL from
 *              the evaluation if the plan has 2^31 - 64 or more far pairs);  2: only
 *              entries with at most 32 of their group's 64 targets, and only with one
 *              right-hand side.  With far_mfma, 0 means 2.
 *   far_split  parts of each group's far list in the group-major kernel, each run by a
 *              wave of its own and summed in part order afterwards (more, shorter waves,
 *              so the last round of waves idles less of the chip): 1 to 4, or 0
 *              (automatic: the fewest parts that give at least twelve rounds of waves at four
 *              waves per SIMD).  Not with far_mfma (0 or 1 only).  stk_plan_tiles reports
 *              the number of parts the evaluation used (1 when every far entry ran
 *              cluster major). */
typedef struct stk_tiles {
    int32_t far_kb;
    int32_t near_kb;
    int32_t near_mfma;
    int32_t far_mfma;
    int32_t far_cm;
    int32_t far_split;
} stk_tiles;
/* Record tiles for (current device's architecture, p, k_rhs, prec); NULL removes the
 * entry.  EINVAL if the tiles do not fit k_rhs and prec. */
stk_status stk_tiles_set(int32_t p, int32_t k_rhs, stk_precision prec, const stk_tiles *tiles);
/* The tiles an evaluation with these parameters would use on the current device;
 * *from_table (may be NULL) is 1 if they come from the table, 0 for the built-in rule. */
stk_status stk_tiles_get(int32_t p, int32_t k_rhs, stk_precision prec, stk_tiles *out, int32_t *from_table);
/* Time every candidate on a synthetic problem of n points uniform in the unit cube
 * (generated on the device; theta and n0 as the caller will use them), record the
 * fastest in the table and return it with its time in ms (either output may be NULL).
 * Allocates and frees its own device memory; synchronises `stream`. */
stk_status stk_autotune(int32_t p, int32_t k_rhs, stk_precision prec, int64_t n, double theta, int32_t n0,
                        stk_tiles *best, double *best_ms, void *stream);
/* Write the table to / merge it from a text file (one "arch p K precision far_kb
 * near_kb near_mfma far_mfma far_cm far_split" line per entry; lines without far_split
 * load as automatic).  Load is all-or-nothing: EINVAL on a malformed or invalid line, and
 * nothing is merged. */
stk_status stk_tiles_save(const char *path);
stk_status stk_tiles_load(const char *path, int32_t *n_entries);
/* The tiles a plan's evaluation used. */
stk_status stk_plan_tiles(const stk_plan *plan, stk_tiles *out);

/* Phase timing, a tracing aid.  While enabled, every entry point records a HIP event
 * on its stream when it starts and after each phase below; stk_profile_read waits for
 * those events, returns the summed milliseconds and the number of timed intervals
 * per phase since the last read (host arrays of STK_NPHASES entries; either may be
 * NULL), and clears the record.  Timing is process-wide; calls on several streams
 * at once are not separated. */
#define STK_NPHASES 10
enum {
    STK_PHASE_TREE = 0,     /* root cube, Morton keys, sort, subdivision, boxes, radii */
    STK_PHASE_MOMENTS = 1,  /* moments, channel blocks, near-field records            */
    STK_PHASE_TARGETS = 2,  /* target keys and sort                                    */
    STK_PHASE_LISTS = 3,    /* MAC traversal: counts, scan, interaction lists          */
    STK_PHASE_NEAR = 4,     /* near-field kernel                                        */
    STK_PHASE_FAR = 5,      /* far-field kernel                                         */
    STK_PHASE_DIRECT = 6,   /* FP64 direct sum                                          */
    STK_PHASE_ADJOINT = 7,  /* adjoint kernels                                          */
    STK_PHASE_FAR_SPARSE = 8, /* far entries applying to few targets, cluster major (K = 1) */
    STK_PHASE_FINISH = 9    /* per-target sums of the near and sparse far partials and of
                               the far field's parts, when it runs in parts                */
};
stk_status stk_profile_enable(int on);
stk_status stk_profile_read(double *ms, int64_t *count);

/* Sizes of a plan's interaction lists: number of 64-target groups, far entries and near
 * entries (each entry is one cluster applied to a subset of one group's targets). */
stk_status stk_plan_info(const stk_plan *plan, int64_t *ngroups, int64_t *n_far_entries, int64_t *n_near_entries);
/* How the plan's far field was split (a scheduling choice, not part of Alg. 1): with one
 * right-hand side, far entries whose lane mask has at most *max_pc bits ran cluster major
 * (*sparse_interactions target-cluster pairs) and the group-major kernel took the rest;
 * *max_pc = 0 means no split.  Either pointer may be NULL. */
stk_status stk_plan_far_split(const stk_plan *plan, int32_t *max_pc, int64_t *sparse_interactions);

void stk_tree_destroy(stk_tree *t);
/* Release a plan.  A plan made by stk_evaluate (it owns its tree) may instead be parked,
 * after a device synchronisation, for reuse by the next stk_evaluate with keep_plan on the
 * same device (at most 2 per device), so that repeated forward + adjoint calls do not
 * allocate device memory; NULL is ignored. */
void stk_plan_destroy(stk_plan *plan);
/* Free the device memory of every parked plan. */
void stk_plan_cache_clear(void);
/* Message for the calling thread's last non-OK status ("" if none). */
const char *stk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STOKESTREE_H */
