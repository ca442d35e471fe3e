// Treecode evaluation (Algorithm 1) for a target set, and the FP64 direct sum.
//
// Targets are sorted into Morton order with the tree's root cube and cut into groups
// of 64 (one wavefront).  A group walks the tree once: at each cluster every lane
// applies the MAC (eq. MAC) to its own target, and the wave splits the cluster into
// the lanes that accept it (a far entry with their mask), the lanes that reach a leaf
// (a near entry) and the lanes that descend (children pushed with their mask).  This
// is exactly Algorithm 1 per target.  The lists are built in one pass into per-group
// slots plus a compaction (two passes, count then fill at the scanned offsets, when the
// slots would not hold them) and kept in the plan for the adjoint.
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>

#include "far_kernels.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {


namespace {

constexpr int STACK = 256;  // >= 1 + 7 * STK_MAX_LEVEL
// per-group list slots of the one-pass traversal: at least these many entries, at most
// this many bytes in all (else two passes)
constexpr int32_t TRAV_SLOT_FAR_MIN = 512, TRAV_SLOT_NEAR_MIN = 256;
constexpr size_t TRAV_SLOT_BYTES_MAX = size_t(2) << 30;

__device__ inline uint64_t rfl64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

struct TravArgs {
    const double *tpos;
    int64_t m;
    const TravNode *node;
    double theta;
    // count pass outputs
    int32_t *gfar, *gnear;              // per group entry counts
    int32_t *cnt_far, *cnt_near, *cnt_pairs;  // per sorted target
    int32_t *gpf, *gpn;                 // per group far (target, cluster) / near (target, leaf) pairs
    // fill pass
    const int32_t *far_off, *near_off;
    int32_t *far_node, *near_node;
    uint64_t *far_mask, *near_mask;
    // one-pass mode: each group's entries at g * slot_far (slot_near) in the slot arrays,
    // at most that many (the counts are exact either way)
    int32_t slot_far, slot_near;
    int32_t *sfar_node, *snear_node;
    uint64_t *sfar_mask, *snear_mask;
};

// COUNT: counts only; FILL: entries at the scanned offsets; SLOT: counts, and entries into
// fixed per-group slots (compacted afterwards)
enum TravMode { TRAV_COUNT = 0, TRAV_FILL = 1, TRAV_SLOT = 2 };

template <int MODE> __global__ __launch_bounds__(64) void k_traverse(TravArgs a) {
    constexpr bool FILL = MODE == TRAV_FILL, SLOT = MODE == TRAV_SLOT;
    __shared__ int32_t st_node[STACK];
    __shared__ uint64_t st_mask[STACK];
    const int32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    const bool valid = t < a.m;
    double x0 = 0, x1 = 0, x2 = 0;
    if (valid) {
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    int32_t nf = 0, nnr = 0, npr = 0;    // per-lane counts
    int32_t fo = 0, no = 0;              // group entry counters
    if (FILL) {
        fo = a.far_off[g];
        no = a.near_off[g];
    }
    int32_t *const sfn = SLOT ? a.sfar_node + int64_t(g) * a.slot_far : nullptr;
    uint64_t *const sfm = SLOT ? a.sfar_mask + int64_t(g) * a.slot_far : nullptr;
    int32_t *const snn = SLOT ? a.snear_node + int64_t(g) * a.slot_near : nullptr;
    uint64_t *const snm = SLOT ? a.snear_mask + int64_t(g) * a.slot_near : nullptr;
    // the node records are read only: through the constant address space the load at the
    // wave-uniform node index stays scalar even in the fill pass, which stores lists
    const STK_CONST_AS TravNode *nodes = (const STK_CONST_AS TravNode *)(a.node);
    const uint64_t vmask = __ballot(valid);
    if (lane == 0) {
        st_node[0] = 0;
        st_mask[0] = vmask;
    }
    int sp = 1;
    __syncthreads();
    while (sp > 0) {
        --sp;
        const int32_t c = __builtin_amdgcn_readfirstlane(st_node[sp]);
        const uint64_t mk = rfl64(st_mask[sp]);
        __syncthreads();
        // the node's whole record in one load: one round trip per visit
        const TravNode nd = nodes[c];
        const double y0 = nd.c[0], y1 = nd.c[1], y2 = nd.c[2], rc = nd.r;
        const int32_t k = nd.nchild, c0 = nd.child0, nc = nd.count;
        // the integer fields are consumed here, so the compiler issues them with the centre
        // and radius instead of sinking their load into the descend branch
        asm volatile("" ::"s"(k), "s"(c0), "s"(nc));
        const bool in = (mk >> lane) & 1ull;
        bool accept = false;
        {
#pragma clang fp contract(off)
            const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
            const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            accept = in && R > 0.0 && rc <= a.theta * R;
        }
        const uint64_t am = __ballot(accept);
        const uint64_t rm = mk & ~am;
        if (am) {
            if (FILL && lane == 0) {
                a.far_node[fo] = c;
                a.far_mask[fo] = am;
            }
            if (SLOT && lane == 0 && fo < a.slot_far) {
                sfn[fo] = c;
                sfm[fo] = am;
            }
            ++fo;
            nf += accept;
        }
        if (rm) {
            if (k == 0) {
                if (FILL && lane == 0) {
                    a.near_node[no] = c;
                    a.near_mask[no] = rm;
                }
                if (SLOT && lane == 0 && no < a.slot_near) {
                    snn[no] = c;
                    snm[no] = rm;
                }
                ++no;
                if ((rm >> lane) & 1ull) {
                    ++nnr;
                    npr += nc;
                }
            } else {
                if (lane == 0)
                    for (int32_t j = k - 1; j >= 0; --j) {
                        st_node[sp + (k - 1 - j)] = c0 + j;
                        st_mask[sp + (k - 1 - j)] = rm;
                    }
                sp += k;
            }
        }
        __syncthreads();
    }
    if (!FILL) {
        int32_t gf = nf, gn = nnr;  // the group's far and near pairs
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            gf += __shfl_xor(gf, o);
            gn += __shfl_xor(gn, o);
        }
        if (lane == 0) {
            a.gfar[g] = fo;
            a.gnear[g] = no;
            a.gpf[g] = gf;
            a.gpn[g] = gn;
        }
        if (valid) {
            a.cnt_far[t] = nf;
            a.cnt_near[t] = nnr;
            a.cnt_pairs[t] = npr;
        }
    }
}

// grid (groups): a group's slot entries to its place in the scanned lists
__global__ __launch_bounds__(256) void k_slot_compact(const int32_t *__restrict__ cnt, const int32_t *__restrict__ off,
                                                      int32_t slot, const int32_t *__restrict__ snode,
                                                      const uint64_t *__restrict__ smask, int32_t *__restrict__ node,
                                                      uint64_t *__restrict__ mask) {
    const int32_t g = blockIdx.x;
    const int32_t n = cnt[g], o = off[g];
    const int64_t base = int64_t(g) * slot;
    for (int32_t j = threadIdx.x; j < n; j += 256) {
        node[o + j] = snode[base + j];
        mask[o + j] = smask[base + j];
    }
}

// ---- target preparation --------------------------------------------------------------
__device__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint64_t quant(double y, double lo, double scale) {
#pragma clang fp contract(off)
    const double v = floor((y - lo) * scale);
    if (!(v > 0.0)) return 0;
    if (v > 2097151.0) return 2097151;
    return (uint64_t)v;
}

__global__ void k_tkeys(const double *__restrict__ pts, int64_t n, double lx, double ly, double lz, double scale,
                        uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t qx = quant(pts[3 * i], lx, scale);
    const uint64_t qy = quant(pts[3 * i + 1], ly, scale);
    const uint64_t qz = quant(pts[3 * i + 2], lz, scale);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    vals[i] = int32_t(i);
}

__global__ void k_gather3(const double *__restrict__ src, const int32_t *__restrict__ perm, int64_t n,
                          double *__restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    dst[3 * i] = src[3 * j];
    dst[3 * i + 1] = src[3 * j + 1];
    dst[3 * i + 2] = src[3 * j + 2];
}

// ---- FP64 direct sum -----------------------------------------------------------------
// grid (target groups, source chunks); each wave sums one chunk of `chunk` consecutive
// sources for 64 targets and writes its partial velocities, which k_direct_reduce adds
// in chunk order
__global__ __launch_bounds__(64) void k_direct(const double *__restrict__ tgt, int64_t m,
                                               const double *__restrict__ src, int64_t n,
                                               const double *__restrict__ f, const double *__restrict__ h,
                                               const double *__restrict__ nu, int32_t chunk,
                                               double *__restrict__ part) {
    const int64_t t = int64_t(blockIdx.x) * 64 + threadIdx.x;
    const bool valid = t < m;
    double x0 = 0, x1 = 0, x2 = 0;
    if (valid) {
        x0 = tgt[3 * t];
        x1 = tgt[3 * t + 1];
        x2 = tgt[3 * t + 2];
    }
    const int64_t j0 = int64_t(blockIdx.y) * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    double u0 = 0, u1 = 0, u2 = 0;
    for (int64_t j = j0; j < j1; ++j) {
        const double d0 = x0 - src[3 * j], d1 = x1 - src[3 * j + 1], d2 = x2 - src[3 * j + 2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double ri = r2 > 0.0 ? rsqrt(r2) : 0.0;
        const double r2i = ri * ri, r3i = ri * r2i;
        const double s = (d0 * f[3 * j] + d1 * f[3 * j + 1] + d2 * f[3 * j + 2]) * r3i;
        const double tt = (d0 * h[3 * j] + d1 * h[3 * j + 1] + d2 * h[3 * j + 2]) *
                          (d0 * nu[3 * j] + d1 * nu[3 * j + 1] + d2 * nu[3 * j + 2]) * (r3i * r2i);
        const double st = s + tt;
        u0 += f[3 * j] * ri + d0 * st;
        u1 += f[3 * j + 1] * ri + d1 * st;
        u2 += f[3 * j + 2] * ri + d2 * st;
    }
    if (valid) {
        double *o = part + (size_t(blockIdx.y) * m + t) * 3;
        o[0] = u0;
        o[1] = u1;
        o[2] = u2;
    }
}

__global__ void k_direct_reduce(const double *__restrict__ part, int64_t m, int nch, double *__restrict__ u) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= 3 * m) return;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[size_t(c) * 3 * m + i];
    u[i] = s;
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// compute units of the current device (looked up once per device)
int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    STK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    STK_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    cus[dev] = n > 0 ? n : 1;
    return cus[dev];
}

// Per (target, right-hand side), when the group-major far field ran in parts: the near
// partials in near-list order (compensated), plus the sparse far partials in their list
// order (compensated; spart may be null), then the far parts in order, written in the
// caller's order.  The arithmetic of a separate near reduction, sparse addition and
// combination, in one pass.
template <typename T>
__global__ void k_finish(const T *__restrict__ npart, const int32_t *__restrict__ ntoff, const T *__restrict__ spart,
                         const int32_t *__restrict__ stoff, const double *__restrict__ fpart, int32_t nsplit,
                         const int32_t *__restrict__ tperm, int64_t m, int32_t K, double *__restrict__ u_out) {
    // right-hand side fastest, so the lanes of a wave read the partials of a target's K
    // right-hand sides, which lie side by side
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m * K) return;
    const int64_t t = i / K, r = i - t * K;
    double un[3];
    {
        Comp<T> acc[3];
        for (int32_t k = ntoff[t]; k < ntoff[t + 1]; ++k)
            for (int q = 0; q < 3; ++q) acc[q].add(npart[(int64_t(k) * K + r) * 3 + q]);
        for (int q = 0; q < 3; ++q) un[q] = acc[q].value();
    }
    if (spart) {
        const int32_t k0 = stoff[t], k1 = stoff[t + 1];
        if (k0 != k1) {
            Comp<T> acc[3];
            for (int32_t k = k0; k < k1; ++k)
                for (int q = 0; q < 3; ++q) acc[q].add(spart[3 * (int64_t(k) * K + r) + q]);
            for (int q = 0; q < 3; ++q) un[q] += acc[q].value();
        }
    }
    double u[3] = {0.0, 0.0, 0.0};
    for (int32_t h = 0; h < nsplit; ++h)
        for (int q = 0; q < 3; ++q) u[q] += fpart[((size_t(h) * K + r) * m + t) * 3 + q];
    const int64_t o = tperm[t];
    for (int q = 0; q < 3; ++q) u_out[(size_t(r) * m + o) * 3 + q] = u[q] + un[q];
}

template <typename T, int KB> void dispatch_far(int p, const FarArgs &a, hipStream_t s) {
    switch (p) {
        case 0: launch_far<0, T, KB>(a, s); break;
        case 1: launch_far<1, T, KB>(a, s); break;
        case 2: launch_far<2, T, KB>(a, s); break;
        case 3: launch_far<3, T, KB>(a, s); break;
        case 4: launch_far<4, T, KB>(a, s); break;
        case 5: launch_far<5, T, KB>(a, s); break;
        case 6: launch_far<6, T, KB>(a, s); break;
        case 7: launch_far<7, T, KB>(a, s); break;
        case 8: launch_far<8, T, KB>(a, s); break;
        case 9: launch_far<9, T, KB>(a, s); break;
        case 10: launch_far<10, T, KB>(a, s); break;
        default: throw Error(STK_EINVAL, "p out of range");
    }
}

}  // namespace

// defined in far_mfma.hpp, instantiated in farm_p*.hip: FP32, K right-hand sides on the
// matrix cores; bm is scratch for the clusters' operand blocks
template <int P> void launch_far_mfma(const FarArgs &a, DBuf &bm, int32_t nn, hipStream_t s);

namespace {

template <typename T, int KB> void dispatch_far_sparse(int p, const FarSparseArgs &a, hipStream_t s) {
    switch (p) {
        case 0: launch_far_sparse<0, T, KB>(a, s); break;
        case 1: launch_far_sparse<1, T, KB>(a, s); break;
        case 2: launch_far_sparse<2, T, KB>(a, s); break;
        case 3: launch_far_sparse<3, T, KB>(a, s); break;
        case 4: launch_far_sparse<4, T, KB>(a, s); break;
        case 5: launch_far_sparse<5, T, KB>(a, s); break;
        case 6: launch_far_sparse<6, T, KB>(a, s); break;
        case 7: launch_far_sparse<7, T, KB>(a, s); break;
        case 8: launch_far_sparse<8, T, KB>(a, s); break;
        case 9: launch_far_sparse<9, T, KB>(a, s); break;
        case 10: launch_far_sparse<10, T, KB>(a, s); break;
        default: throw Error(STK_EINVAL, "p out of range");
    }
}

// per (target, right-hand side): its cluster-major far velocities in list order,
// compensated, added to unear (m,K,3)
template <typename T>
__global__ void k_cm_add(const T *__restrict__ part, const int32_t *__restrict__ toff, int64_t m, int32_t K,
                         double *__restrict__ unear) {
    const int64_t tr = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tr >= m * K) return;
    const int64_t t = tr / K;
    const int32_t k0 = toff[t], k1 = toff[t + 1];
    if (k0 == k1) return;
    const int64_t r = tr - t * K;
    Comp<T> acc[3];
    for (int32_t k = k0; k < k1; ++k)
        for (int q = 0; q < 3; ++q) acc[q].add(part[3 * (int64_t(k) * K + r) + q]);
    for (int q = 0; q < 3; ++q) unear[3 * tr + q] += acc[q].value();
}

void dispatch_far_mfma(int p, const FarArgs &a, DBuf &bm, int32_t nn, hipStream_t s) {
    switch (p) {
        case 0: launch_far_mfma<0>(a, bm, nn, s); break;
        case 1: launch_far_mfma<1>(a, bm, nn, s); break;
        case 2: launch_far_mfma<2>(a, bm, nn, s); break;
        case 3: launch_far_mfma<3>(a, bm, nn, s); break;
        case 4: launch_far_mfma<4>(a, bm, nn, s); break;
        case 5: launch_far_mfma<5>(a, bm, nn, s); break;
        case 6: launch_far_mfma<6>(a, bm, nn, s); break;
        case 7: launch_far_mfma<7>(a, bm, nn, s); break;
        case 8: launch_far_mfma<8>(a, bm, nn, s); break;
        case 9: launch_far_mfma<9>(a, bm, nn, s); break;
        case 10: launch_far_mfma<10>(a, bm, nn, s); break;
        default: throw Error(STK_EINVAL, "p out of range");
    }
}

}  // namespace

namespace {
CmInput far_cm_input(Plan &pl, int max_pc) {
    return CmInput{pl.far_off.as<int32_t>(), pl.far_node.as<int32_t>(), pl.far_mask.as<uint64_t>(), pl.n_far_entries,
                   pl.ngroups, pl.m, max_pc, max_pc >= 64 ? pl.cnt_far.as<int32_t>() : nullptr};
}
CmInput near_cm_input(Plan &pl) {
    return CmInput{pl.near_off.as<int32_t>(), pl.near_node.as<int32_t>(), pl.near_mask.as<uint64_t>(),
                   pl.n_near_entries, pl.ngroups, pl.m, 64, pl.cnt_near.as<int32_t>()};
}
}  // namespace

void far_sparse(Tree &t, Plan &pl, double *unear, int max_pc, hipStream_t s, bool add) {
    const CmInput in = far_cm_input(pl, max_pc);
    cm_stage1(t, pl.fcm, in, s);
    cm_stage2(t, pl.fcm, in, s);
    cm_stage3(t, pl.fcm, in, s);
    far_sparse_run(t, pl, unear, max_pc, s, add);
}

void far_sparse_run(Tree &t, Plan &pl, double *unear, int max_pc, hipStream_t s, bool add) {
    (void)max_pc;
    const int64_t m = pl.m;
    const int K = t.k_rhs;
    ClusterMajor &cm = pl.fcm;
    const size_t tsz = t.prec == STK_FP64 ? sizeof(double) : sizeof(float);
    void *part = reserve<unsigned char>(cm.part, tsz * 3 * size_t(K) * size_t(cm.n_inc) + tsz);
    FarSparseArgs sa{pl.tpos_p, cm.item_node.as<int32_t>(), cm.item_i0.as<int32_t>(),
                     cm.item_i1.as<int32_t>(), cm.inc_tgt.as<int32_t>(), cm.inc_slot.as<int32_t>(),
                     t.ncenter.as<double>(), t.nrho.as<double>(), t.wblk.p, part, cm.n_items, K};
    const int kb = pl.tiles.far_kb;
    if (t.prec == STK_FP64)
        dispatch_far_sparse<double, 1>(t.p, sa, s);
    else if (kb == 4)
        dispatch_far_sparse<float, 4>(t.p, sa, s);
    else if (kb == 2)
        dispatch_far_sparse<float, 2>(t.p, sa, s);
    else
        dispatch_far_sparse<float, 1>(t.p, sa, s);
    if (add && m > 0 && cm.n_inc > 0) {
        if (t.prec == STK_FP64)
            hipLaunchKernelGGL(k_cm_add<double>, dim3(nblk(m * K, 256)), dim3(256), 0, s,
                               static_cast<const double *>(part), cm.toff.as<int32_t>(), m, K, unear);
        else
            hipLaunchKernelGGL(k_cm_add<float>, dim3(nblk(m * K, 256)), dim3(256), 0, s,
                               static_cast<const float *>(part), cm.toff.as<int32_t>(), m, K, unear);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_FAR_SPARSE, s);
}

Plan::~Plan() {
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (owns_tree) delete tree;
}

void build_lists(Tree &t, Plan &pl, const double *tgt, int64_t m, double theta, bool same_as_sources,
                 hipStream_t s) {
    pl.tree = &t;
    pl.m = m;
    pl.theta = theta;
    const int32_t ng = int32_t((m + 63) / 64);
    pl.ngroups = ng;
    prof_mark(-1, s);

    // targets in Morton order of the tree's root cube
    if (same_as_sources) {
        pl.tperm_p = t.perm.as<int32_t>();
        pl.tpos_p = t.pos.as<double>();
    } else {
        int32_t *tperm = reserve<int32_t>(pl.tperm, size_t(m));
        double *tpos = reserve<double>(pl.tpos, size_t(m) * 3);
        pl.tperm_p = tperm;
        pl.tpos_p = tpos;
        uint64_t *keys = reserve<uint64_t>(t.s_keys, size_t(m));
        hipLaunchKernelGGL(k_tkeys, dim3(nblk(m, 256)), dim3(256), 0, s, tgt, m, t.lo[0], t.lo[1], t.lo[2],
                           t.scale, keys, tperm);
        STK_CHECK_LAUNCH();
        radix_sort_pairs(t, keys, tperm, m, 63, s);
        hipLaunchKernelGGL(k_gather3, dim3(nblk(m, 256)), dim3(256), 0, s, tgt, tperm, m, tpos);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_TARGETS, s);

    // interaction lists: count, scan, fill
    TravArgs ta{};
    ta.tpos = pl.tpos_p;
    ta.m = m;
    ta.node = t.trav.as<TravNode>();
    ta.theta = theta;
    int32_t *gcnt = reserve<int32_t>(t.s_vals, size_t(ng) * 4);
    ta.gfar = gcnt;
    ta.gnear = gcnt + ng;
    ta.gpf = gcnt + 2 * size_t(ng);
    ta.gpn = gcnt + 3 * size_t(ng);
    ta.cnt_far = reserve<int32_t>(pl.cnt_far, size_t(m));
    ta.cnt_near = reserve<int32_t>(pl.cnt_near, size_t(m));
    ta.cnt_pairs = reserve<int32_t>(pl.cnt_pairs, size_t(m));
    // One pass when the per-group slots fit: the traversal counts and writes each group's
    // entries into slots sized from the longest lists of the tree's last evaluation (plus a
    // quarter; at least 512 far and 256 near entries), which are then compacted into the
    // scanned lists.  If a group overflowed its slots, a second pass writes the lists at the
    // scanned offsets, as the two-pass build always does when the slots would not fit.
    const int32_t sf = std::max(t.slot_far, TRAV_SLOT_FAR_MIN), sn = std::max(t.slot_near, TRAV_SLOT_NEAR_MIN);
    const bool one_pass = ng > 0 && size_t(ng) * size_t(sf + sn) * 12 <= TRAV_SLOT_BYTES_MAX;
    if (one_pass) {
        unsigned char *sb = reserve<unsigned char>(t.s_slot, size_t(ng) * size_t(sf + sn) * 12);
        ta.slot_far = sf;
        ta.slot_near = sn;
        ta.sfar_mask = reinterpret_cast<uint64_t *>(sb);
        ta.snear_mask = ta.sfar_mask + size_t(ng) * sf;
        ta.sfar_node = reinterpret_cast<int32_t *>(ta.snear_mask + size_t(ng) * sn);
        ta.snear_node = ta.sfar_node + size_t(ng) * sf;
        hipLaunchKernelGGL(k_traverse<TRAV_SLOT>, dim3(ng), dim3(64), 0, s, ta);
    } else {
        hipLaunchKernelGGL(k_traverse<TRAV_COUNT>, dim3(ng), dim3(64), 0, s, ta);
    }
    STK_CHECK_LAUNCH();
    long long *inc_d = reserve<long long>(pl.far_inc, 4);
    int32_t *foff = reserve<int32_t>(pl.far_off, size_t(ng) + 1);
    int32_t *noff = reserve<int32_t>(pl.near_off, size_t(ng) + 1);
    // list offsets, pair totals and the longest group lists
    scan2_stats(ta.gfar, foff, ta.gnear, noff, ta.gpf, ta.gpn, ng, inc_d, t.s_scan, s);
    int32_t tot[2];
    int64_t inc[2], longest[2];
    {
        const PeekSrc src[6] = {{foff + ng, 4}, {noff + ng, 4}, {inc_d, 8}, {inc_d + 1, 8}, {inc_d + 2, 8},
                                {inc_d + 3, 8}};
        int64_t v[6];
        peek(t.peek, s, 6, src, v);
        tot[0] = int32_t(v[0]);
        tot[1] = int32_t(v[1]);
        inc[0] = v[2];
        inc[1] = v[3];
        longest[0] = v[4];
        longest[1] = v[5];
    }
    pl.n_far_entries = tot[0];
    pl.n_near_entries = tot[1];
    pl.n_far_inc = int64_t(inc[0]);
    // the near field always runs on its cluster-major (leaf-major) view
    if (int64_t(inc[1]) >= CM_MAX_INC)
        throw Error(STK_EINVAL, "too many near-field (target, leaf) pairs for the leaf-major lists");
    ta.far_off = foff;
    ta.near_off = noff;
    ta.far_node = reserve<int32_t>(pl.far_node, size_t(tot[0]) + 1);
    ta.far_mask = reserve<uint64_t>(pl.far_mask, size_t(tot[0]) + 1);
    ta.near_node = reserve<int32_t>(pl.near_node, size_t(tot[1]) + 1);
    ta.near_mask = reserve<uint64_t>(pl.near_mask, size_t(tot[1]) + 1);
    if (one_pass && longest[0] <= sf && longest[1] <= sn) {
        hipLaunchKernelGGL(k_slot_compact, dim3(ng), dim3(256), 0, s, ta.gfar, foff, sf, ta.sfar_node, ta.sfar_mask,
                           ta.far_node, ta.far_mask);
        STK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_slot_compact, dim3(ng), dim3(256), 0, s, ta.gnear, noff, sn, ta.snear_node,
                           ta.snear_mask, ta.near_node, ta.near_mask);
        STK_CHECK_LAUNCH();
    } else if (ng > 0) {
        hipLaunchKernelGGL(k_traverse<TRAV_FILL>, dim3(ng), dim3(64), 0, s, ta);
        STK_CHECK_LAUNCH();
    }
    t.slot_far = int32_t(std::min<int64_t>(longest[0] + longest[0] / 4 + 1, INT32_MAX / 2));
    t.slot_near = int32_t(std::min<int64_t>(longest[1] + longest[1] / 4 + 1, INT32_MAX / 2));
}

void evaluate(Tree &t, Plan &pl, const double *tgt, int64_t m, double theta, double *u_out, bool same_as_sources,
              hipStream_t s) {
    pl.reg_eps = -1.0;
    build_lists(t, pl, tgt, m, theta, same_as_sources, s);
    const int32_t ng = pl.ngroups;
    const double *tpos = pl.tpos_p;
    const int32_t *tperm = pl.tperm_p;
    const int32_t *foff = pl.far_off.as<int32_t>();

    // kernel variants: right-hand sides per pass, matrix cores
    const int K = t.k_rhs;
    pl.tiles = pl.forced ? pl.force : tiles_for(t.p, K, t.prec);
    if (!tiles_valid(pl.tiles, K, t.prec)) throw Error(STK_EINVAL, "kernel tiles do not fit this evaluation");
    const int kb = pl.tiles.far_kb;

    // far entries that apply to few targets of their group (one right-hand side), or every
    // far entry (tile far_cm, or automatically when the group lists' lanes are mostly
    // idle), run cluster major (their velocities are added to the near part); the
    // group-major kernel skips them
    const double util = pl.n_far_entries > 0 ? double(pl.n_far_inc) / (64.0 * double(pl.n_far_entries)) : 1.0;
    const bool cm_fits = pl.n_far_inc < CM_MAX_INC;
    const bool all_cm = !pl.tiles.far_mfma && cm_fits &&
                        (pl.tiles.far_cm == FAR_CM_ON || (pl.tiles.far_cm == FAR_CM_AUTO && util < FAR_CM_UTIL));
    if (pl.tiles.far_cm == FAR_CM_ON && !cm_fits)
        throw Error(STK_EINVAL, "far_cm: too many far interactions for the cluster-major lists");
    const int sparse_max = all_cm ? 64 : (K == 1 && cm_fits ? FAR_SPARSE_MAX : 0);
    pl.far_sparse_max = sparse_max;
    // parts of each group's far list (tile far_split; automatically enough parts for
    // FAR_SPLIT_ROUNDS rounds of waves, so the last round idles little of the chip)
    int32_t nsplit = 1;
    if (!all_cm && !pl.tiles.far_mfma && ng > 0) {
        if (pl.tiles.far_split > 0) {
            nsplit = pl.tiles.far_split;
        } else {
            const int64_t slots = int64_t(device_cus()) * 4 * 4;
            while (nsplit < FAR_SPLIT_MAX && int64_t(ng) * nsplit < FAR_SPLIT_ROUNDS * slots) ++nsplit;
        }
    }
    pl.tiles.far_split = nsplit;
    // with the far field in parts, one final pass adds the near partials, the sparse far
    // partials and the parts; otherwise the near part is reduced into unear, the sparse
    // partials added to it, and the far kernel adds it
    const bool finish = nsplit > 1 && m > 0;

    // The near field's leaf-major view and the sparse far entries' cluster-major view (each
    // a chain of small sorts and scans with host readbacks between them, and each with its
    // own scratch): on two streams when the plan names a second one, their stages
    // interleaved so that one view's kernels run while the host waits for the other's
    // readback.  Then the near field, then the far field.
    double *unear = reserve<double>(t.s_tmp, size_t(m) * K * 3);
    const bool two = sparse_max > 0 && pl.aux && pl.aux != s;
    hipStream_t s3 = two ? pl.aux : s;
    if (two) {
        for (hipEvent_t &e : pl.ev)
            if (!e) STK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        STK_HIP(hipEventRecord(pl.ev[0], s));  // the lists
        STK_HIP(hipStreamWaitEvent(s3, pl.ev[0], 0));
    }
    const CmInput nin = near_cm_input(pl), fin = far_cm_input(pl, sparse_max);
    cm_stage1(t, pl.ncm, nin, s);
    if (sparse_max > 0) cm_stage1(t, pl.fcm, fin, s3);
    cm_stage2(t, pl.ncm, nin, s);
    if (sparse_max > 0) cm_stage2(t, pl.fcm, fin, s3);
    cm_stage3(t, pl.ncm, nin, s);
    prof_mark(STK_PHASE_LISTS, s);
    if (sparse_max > 0) {
        cm_stage3(t, pl.fcm, fin, s3);
        if (two) STK_HIP(hipEventRecord(pl.ev[1], s3));  // the sparse far entries' view
    }
    near_kernels(t, pl, unear, s, !finish);
    // moments computed beside the lists and the near field (on another stream) must be
    // complete from here on: the far kernels read the clusters' streams
    if (pl.moments_ready) {
        STK_HIP(hipStreamWaitEvent(s, pl.moments_ready, 0));
        pl.moments_ready = nullptr;
    }
    if (sparse_max > 0) {
        if (two) STK_HIP(hipStreamWaitEvent(s, pl.ev[1], 0));
        far_sparse_run(t, pl, unear, sparse_max, s, !finish);
    }
    double *fpart = nsplit > 1 ? reserve<double>(pl.far_part, size_t(nsplit) * K * size_t(m) * 3) : nullptr;
    FarArgs fa{tpos, m, foff, pl.far_node.as<int32_t>(), pl.far_mask.as<uint64_t>(), t.ncenter.as<double>(),
               t.nrho.as<double>(), t.wblk.p, unear, tperm, u_out, ng, K, sparse_max, nsplit, fpart};
    if (t.prec == STK_FP64)
        dispatch_far<double, 1>(t.p, fa, s);
    else if (pl.tiles.far_mfma)
        dispatch_far_mfma(t.p, fa, t.s_bm, t.nnodes, s);
    else if (kb == 4)
        dispatch_far<float, 4>(t.p, fa, s);
    else if (kb == 2)
        dispatch_far<float, 2>(t.p, fa, s);
    else
        dispatch_far<float, 1>(t.p, fa, s);
    prof_mark(STK_PHASE_FAR, s);
    if (finish) {
        const ClusterMajor &nc = pl.ncm, &fc = pl.fcm;
        const int32_t *stoff = sparse_max > 0 ? fc.toff.as<int32_t>() : nullptr;
        if (t.prec == STK_FP64)
            hipLaunchKernelGGL(k_finish<double>, dim3(nblk(m * K, 256)), dim3(256), 0, s, nc.part.as<double>(),
                               nc.toff.as<int32_t>(), sparse_max > 0 ? fc.part.as<double>() : nullptr, stoff, fpart,
                               nsplit, tperm, m, K, u_out);
        else
            hipLaunchKernelGGL(k_finish<float>, dim3(nblk(m * K, 256)), dim3(256), 0, s, nc.part.as<float>(),
                               nc.toff.as<int32_t>(), sparse_max > 0 ? fc.part.as<float>() : nullptr, stoff, fpart,
                               nsplit, tperm, m, K, u_out);
        STK_CHECK_LAUNCH();
        prof_mark(STK_PHASE_FINISH, s);
    }
}

DirectShape direct_shape(int64_t m, int64_t n) {
    // about DIRECT_WAVES (target group, chunk) waves when the targets are few, so a
    // sampled-target reference still fills the chip; at most DIRECT_CHUNK_MAX sources per
    // wave (the partial buffer stays 3 m ceil(n / 8192) doubles for large m)
    constexpr int64_t DIRECT_WAVES = 32768, DIRECT_CHUNK_MIN = 512, DIRECT_CHUNK_MAX = 8192;
    const int64_t ng = (m + 63) / 64;
    const int64_t want = (DIRECT_WAVES + ng - 1) / ng;
    int64_t c = (n + want - 1) / want;
    c = (c + 255) / 256 * 256;
    c = c < DIRECT_CHUNK_MIN ? DIRECT_CHUNK_MIN : (c > DIRECT_CHUNK_MAX ? DIRECT_CHUNK_MAX : c);
    DirectShape d;
    d.chunk = int32_t(c);
    d.nch = int32_t((n + c - 1) / c);
    return d;
}

void direct_launch(const double *tgt, int64_t m, const double *src, int64_t n, const double *f, const double *h,
                   const double *nu, const DirectShape &d, double *part, double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_direct, dim3(nblk(m, 64), unsigned(d.nch)), dim3(64), 0, s, tgt, m, src, n, f, h, nu,
                       d.chunk, part);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_direct_reduce, dim3(nblk(3 * m, 256)), dim3(256), 0, s, part, m, d.nch, u);
    STK_CHECK_LAUNCH();
}

void direct_sum(const double *tgt, int64_t m, const double *src, int64_t n, const double *f, const double *h,
                const double *nu, int32_t K, double *u_out, hipStream_t s) {
    const DirectShape d = direct_shape(m, n);
    double *part = nullptr;
    prof_mark(-1, s);
    STK_HIP(hipMallocAsync((void **)&part, sizeof(double) * 3 * size_t(m) * d.nch, s));
    for (int r = 0; r < K; ++r)
        direct_launch(tgt, m, src, n, f + size_t(r) * n * 3, h + size_t(r) * n * 3, nu, d, part,
                      u_out + size_t(r) * m * 3, s);
    prof_mark(STK_PHASE_DIRECT, s);
    STK_HIP(hipFreeAsync(part, s));
}

}  // namespace stk
