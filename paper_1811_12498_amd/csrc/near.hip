// Near field (Alg. 1: leaves that fail eq. MAC are summed directly with the contracted
// pair of Sec. 4.1), leaf major.
//
// The traversal leaves group-major lists: for each group of 64 Morton-consecutive
// targets, entries (leaf, lane mask).  A wave that walked those entries would idle every
// lane whose target does not need the leaf.  Instead the entries are transposed: every
// (target, near leaf) incidence is placed in a leaf-sorted array, and each work item is
// one leaf with up to 64 of its targets, so every lane of an item has work.  An item's
// wave reads the leaf's source records through the scalar cache (wave-uniform) and
// writes one partial velocity per incidence to the slot that incidence has in its
// target's near list; a per-target pass then adds the partials in list order with the
// compensated accumulator.  The result is the same, bit for bit, as a walk of the
// target's own near list.
#include "far_kernels.hpp"
#include "lists.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {
namespace {

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// One source's contribution (contracted pair of Sec. 4.1), arranged as
//   u_i += (1/r) (f_i + d_i s),   s = (d.f + (d.h)(d.nu)/r^2) / r^2,
// which is f_i/r + d_i (d.f)/r^3 + d_i (d.h)(d.nu)/r^5, in two FMAs per component,
// for KB right-hand sides that share the geometry (d, r, d.nu).  g = (y, nu) and
// w[r] = (f, h) are wave-uniform (held in SGPRs).  CHECK: a pair with r = 0 may occur
// (the coincident source is skipped, Sec. 2); without it the caller has shown that
// every pair of the leaf is at distance > 1e-15.
template <bool CHECK, int KB>
__device__ inline void pair_f64(double x0, double x1, double x2, const double g[6], const double (*w)[6],
                                double (*u)[3]) {
    const double d0 = x0 - g[0], d1 = x1 - g[1], d2 = x2 - g[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    double ri = rsqrt(r2);
    if constexpr (CHECK) ri = r2 > 0.0 ? ri : 0.0;
    const double r2i = ri * ri;
    const double dn = d0 * g[3] + d1 * g[4] + d2 * g[5];
#pragma unroll
    for (int r = 0; r < KB; ++r) {
        const double df = d0 * w[r][0] + d1 * w[r][1] + d2 * w[r][2];
        const double dh = d0 * w[r][3] + d1 * w[r][4] + d2 * w[r][5];
        const double sc = fma(dh, dn * r2i, df) * r2i;
        u[r][0] = fma(ri, fma(d0, sc, w[r][0]), u[r][0]);
        u[r][1] = fma(ri, fma(d1, sc, w[r][1]), u[r][1]);
        u[r][2] = fma(ri, fma(d2, sc, w[r][2]), u[r][2]);
    }
}

// Mixed precision: d = x - y and d.nu in FP64 (on a surface with nu the normal d.nu is
// O(|d|^2), so its absolute rounding must stay at FP64 level), the rest in FP32.
template <bool CHECK, int KB>
__device__ inline void pair_mixed(double x0, double x1, double x2, const double g[6], const float (*w)[6],
                                  float (*u)[3]) {
    const double d0 = x0 - g[0], d1 = x1 - g[1], d2 = x2 - g[2];
    const double dn = d0 * g[3] + d1 * g[4] + d2 * g[5];
    const float f0 = float(d0), f1 = float(d1), f2 = float(d2);
    const float r2 = f0 * f0 + f1 * f1 + f2 * f2;
    float ri = __frsqrt_rn(r2);
    if constexpr (CHECK) ri = r2 > 0.0f ? ri : 0.0f;
    const float r2i = ri * ri;
    const float q = float(dn) * r2i;
#pragma unroll
    for (int r = 0; r < KB; ++r) {
        const float df = f0 * w[r][0] + f1 * w[r][1] + f2 * w[r][2];
        const float dh = f0 * w[r][3] + f1 * w[r][4] + f2 * w[r][5];
        const float sc = fmaf(dh, q, df) * r2i;
        u[r][0] = fmaf(ri, fmaf(f0, sc, w[r][0]), u[r][0]);
        u[r][1] = fmaf(ri, fmaf(f1, sc, w[r][1]), u[r][1]);
        u[r][2] = fmaf(ri, fmaf(f2, sc, w[r][2]), u[r][2]);
    }
}

// sum over sources [s, s + n) of one leaf for KB right-hand sides; wr points at source
// 0's weights of the first of them and ws is the per-source stride (both wave-uniform).
// The records are walked with uniform pointers advanced once per batch of NBATCH
// sources, read at constant offsets (WS = ws known at compile time when the call has
// exactly KB right-hand sides; 0 = the runtime stride), so the scalar loads of a batch
// merge into a few wide ones and no address is rebuilt per source.
template <typename T, bool CHECK, int KB, int WS>
__device__ inline void near_leaf(const double *__restrict__ geo_g, const T *__restrict__ wr_g, int ws, int32_t s,
                                 int32_t n, double x0, double x1, double x2, T (*u)[3]) {
    constexpr int NBATCH = KB == 1 ? 4 : (KB == 2 ? 2 : 1);
    const int wstride = WS ? WS : ws;
    // the records are not written while the kernel runs: read them as constant memory, so
    // the partial stores between right-hand-side blocks do not turn them into vector loads
    const STK_CONST_AS double *g = (const STK_CONST_AS double *)(geo_g) + 6 * int64_t(s);
    const STK_CONST_AS T *w = (const STK_CONST_AS T *)(wr_g) + int64_t(s) * wstride;
    int32_t left = n;
    // a batch's records as single aggregates (one base address, merged wide loads)
    struct GeoBatch {
        double v[NBATCH][6];
    };
    struct WtsBatch {
        T v[NBATCH][KB][6];
    };
    for (; left >= NBATCH; left -= NBATCH, g += 6 * NBATCH, w += NBATCH * wstride) {
        double gb[NBATCH][6];
        T wb[NBATCH][KB][6];
        {
            const GeoBatch gg = *(const STK_CONST_AS GeoBatch *)g;
#pragma unroll
            for (int b = 0; b < NBATCH; ++b)
#pragma unroll
                for (int q = 0; q < 6; ++q) gb[b][q] = gg.v[b][q];
        }
        if constexpr (WS == 6 * KB) {
            const WtsBatch ww = *(const STK_CONST_AS WtsBatch *)w;
#pragma unroll
            for (int b = 0; b < NBATCH; ++b)
#pragma unroll
                for (int r = 0; r < KB; ++r)
#pragma unroll
                    for (int q = 0; q < 6; ++q) wb[b][r][q] = ww.v[b][r][q];
        } else {
#pragma unroll
            for (int b = 0; b < NBATCH; ++b)
#pragma unroll
                for (int r = 0; r < KB; ++r)
#pragma unroll
                    for (int q = 0; q < 6; ++q) wb[b][r][q] = w[b * wstride + 6 * r + q];
        }
#pragma unroll
        for (int b = 0; b < NBATCH; ++b) {
            if constexpr (sizeof(T) == 8)
                pair_f64<CHECK, KB>(x0, x1, x2, gb[b], reinterpret_cast<const double(*)[6]>(wb[b]),
                                    reinterpret_cast<double(*)[3]>(u));
            else
                pair_mixed<CHECK, KB>(x0, x1, x2, gb[b], reinterpret_cast<const float(*)[6]>(wb[b]),
                                      reinterpret_cast<float(*)[3]>(u));
        }
    }
    for (; left > 0; --left, g += 6, w += wstride) {
        double gc[6];
        T wc[KB][6];
#pragma unroll
        for (int q = 0; q < 6; ++q) gc[q] = g[q];
#pragma unroll
        for (int r = 0; r < KB; ++r)
#pragma unroll
            for (int q = 0; q < 6; ++q) wc[r][q] = w[6 * r + q];
        if constexpr (sizeof(T) == 8)
            pair_f64<CHECK, KB>(x0, x1, x2, gc, reinterpret_cast<const double(*)[6]>(wc),
                                reinterpret_cast<double(*)[3]>(u));
        else
            pair_mixed<CHECK, KB>(x0, x1, x2, gc, reinterpret_cast<const float(*)[6]>(wc),
                                  reinterpret_cast<float(*)[3]>(u));
    }
}

// squared distance from x to the closed box [lo, hi] (FP64)
__device__ inline double box_dist2(double x0, double x1, double x2, const double *lo, const double *hi) {
    const double e0 = fmax(fmax(lo[0] - x0, x0 - hi[0]), 0.0);
    const double e1 = fmax(fmax(lo[1] - x1, x1 - hi[1]), 0.0);
    const double e2 = fmax(fmax(lo[2] - x2, x2 - hi[2]), 0.0);
    return e0 * e0 + e1 * e1 + e2 * e2;
}

// ---- cluster-major view of group lists ---------------------------------------------------
// an entry is kept iff its mask has at most max_pc bits
__device__ inline bool kept(uint64_t mk, int max_pc) { return __popcll(mk) <= max_pc; }

// sort keys: the node of a kept entry, nn (after every node) for the others
__global__ void k_cm_keys(const int32_t *__restrict__ node, const uint64_t *__restrict__ mask, int64_t ne, int32_t nn,
                          int max_pc, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    keys[e] = kept(mask[e], max_pc) ? uint64_t(node[e]) : uint64_t(nn);
    vals[e] = int32_t(e);
}

// compaction of the kept entries (when most are dropped): flags, then (node, entry) pairs
__global__ void k_cm_flag(const uint64_t *__restrict__ mask, int64_t ne, int max_pc, int32_t *__restrict__ flag) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    flag[e] = kept(mask[e], max_pc) ? 1 : 0;
}
__global__ void k_cm_compact(const int32_t *__restrict__ node, const uint64_t *__restrict__ mask, int64_t ne,
                             int max_pc, const int32_t *__restrict__ fpos, uint64_t *__restrict__ keys,
                             int32_t *__restrict__ vals) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= ne || !kept(mask[e], max_pc)) return;
    keys[fpos[e]] = uint64_t(node[e]);
    vals[fpos[e]] = int32_t(e);
}

// sorted entry k: its incidences (0 if not kept); pos[e] = sorted position of entry e
__global__ void k_cm_pos(const int32_t *__restrict__ ent, const uint64_t *__restrict__ mask, int64_t ne, int max_pc,
                         int32_t *__restrict__ pc, int32_t *__restrict__ pos) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= ne) return;
    const int32_t e = ent[k];
    const uint64_t mk = mask[e];
    pc[k] = kept(mk, max_pc) ? __popcll(mk) : 0;
    pos[e] = int32_t(k);
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
    return (uint64_t(uint32_t(__shfl(int(v >> 32), src, 64))) << 32) | uint32_t(__shfl(int(uint32_t(v)), src, 64));
}
__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    return (uint64_t(uint32_t(__shfl_xor(int(v >> 32), m, 64))) << 32) |
           uint32_t(__shfl_xor(int(uint32_t(v)), m, 64));
}

// 64 x 64 bit transpose over a wave (every lane calls it): lane j holds row j; on return
// lane l holds column l, whose bit j is bit l of row j.  Six steps, each swapping the
// off-diagonal blocks of half the previous size between lanes s apart.
__device__ inline uint64_t wave_transpose64(uint64_t row) {
    const int lane = threadIdx.x & 63;
    constexpr uint64_t keep[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                  0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int s = 32 >> k;
        const uint64_t p = shfl_xor_u64(row, s), m = keep[k];
        row = (lane & s) == 0 ? ((row & m) | ((p & m) << s)) : ((row & ~m) | ((p & ~m) >> s));
    }
    return row;
}

// per target: number of kept entries of its group that apply to it.  The group's masks are
// read 64 at a time, one per lane; the transposed bit matrix gives each lane the entries
// that include its target.
__global__ __launch_bounds__(64) void k_cm_tcount(const int32_t *__restrict__ off, const uint64_t *__restrict__ mask,
                                                  int64_t m, int max_pc, int32_t *__restrict__ tcnt) {
    const int32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    int32_t c = 0;
    const int32_t e0 = off[g], e1 = off[g + 1];
    for (int32_t eb = e0; eb < e1; eb += 64) {
        const int nb = e1 - eb < 64 ? e1 - eb : 64;
        const uint64_t mj = lane < nb ? mask[eb + lane] : 0ull;
        const uint64_t kb = __ballot(lane < nb && kept(mj, max_pc));
        c += __popcll(wave_transpose64(mj) & kb);
    }
    if (t < m) tcnt[t] = c;
}

// per node c in [0, nn]: its first sorted entry eoff[c] (the first key >= c) and first
// incidence loff[c]; for c < nn also its number of items of up to `per` incidences
__global__ void k_cm_nodes(const uint64_t *__restrict__ keys, int64_t nk, int32_t nn,
                           const int32_t *__restrict__ incoff, int32_t per, int32_t *__restrict__ eoff,
                           int32_t *__restrict__ loff, int32_t *__restrict__ icnt) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nn) return;
    auto first = [&](int32_t v) {
        int64_t lo = 0, hi = nk;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < uint64_t(v))
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    };
    const int64_t e0 = first(c);
    const int32_t l0 = incoff[e0];
    eoff[c] = int32_t(e0);
    loff[c] = l0;
    if (c < nn) icnt[c] = (incoff[first(c + 1)] - l0 + per - 1) / per;
}

// one wave per group: lane l walks the group's kept entries that include its target, in
// list order, and places each incidence (target, slot) at its node-major position.  The
// entries are read 64 at a time, one per lane (mask, and the first incidence of a kept
// entry); the transposed bit matrix gives each lane its entries of the batch.
__global__ __launch_bounds__(64) void k_cm_fill(const int32_t *__restrict__ off, const uint64_t *__restrict__ mask,
                                                int max_pc, const int32_t *__restrict__ pos,
                                                const int32_t *__restrict__ incoff, const int32_t *__restrict__ toff,
                                                int64_t m, int32_t *__restrict__ inc_tgt,
                                                int32_t *__restrict__ inc_slot) {
    const int32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t slot = t < m ? toff[t] : 0;
    const int32_t e0 = off[g], e1 = off[g + 1];
    for (int32_t eb = e0; eb < e1; eb += 64) {
        const int nb = e1 - eb < 64 ? e1 - eb : 64;
        uint64_t mj = 0ull;
        int32_t pj = 0;
        if (lane < nb) {
            mj = mask[eb + lane];
            pj = pos[eb + lane];
        }
        const bool kj = lane < nb && kept(mj, max_pc);
        // an entry that is not kept has no sorted position: its lane reads incoff[0] and
        // the value is not used
        const int32_t ij = incoff[kj ? pj : 0];
        uint64_t mine = wave_transpose64(mj) & __ballot(kj);
        while (__ballot(mine != 0ull) != 0ull) {  // every lane takes part in the shuffles
            const bool have = mine != 0ull;
            const int j = have ? __builtin_ctzll(mine) : 0;
            mine &= mine - 1ull;
            const uint64_t mk = shfl_u64(mj, j);
            const int32_t io = __shfl(ij, j, 64);
            if (have) {
                const int32_t q = io + __popcll(mk & lt);
                inc_tgt[q] = int32_t(t);
                inc_slot[q] = slot++;
            }
        }
    }
}

// ---- kernels ---------------------------------------------------------------------------
struct NearArgs {
    const double *tpos;                    // (m,3) sorted targets
    const int32_t *item_leaf, *item_i0, *item_i1;
    const int32_t *inc_tgt, *inc_slot;
    const int32_t *start, *count;          // leaf source ranges
    const double *bmin, *bmax;             // (nn,3) tight source boxes
    const double *geo;                     // (n,6) y, nu
    const void *wts;                       // (n,K,6) f, h in T
    void *part;                            // (incidences, K, 3) T
    int32_t nitems;
    int32_t K;                             // right-hand sides (a multiple of KB)
    double eps2 = 0.0;                     // regularized kernels: eps^2
};

// one wave per item: the item's leaf against up to 64 of its targets, for all right-hand
// sides in blocks of KB.  Items of one leaf are consecutive and go to one XCD, so the
// leaf's records are shared in its L2.
template <typename T, int KB> __global__ __launch_bounds__(64) void k_near(NearArgs a) {
    const int32_t it = xcd_item<XCD_CHUNK_NEAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int32_t c = a.item_leaf[it];
    const int32_t i0 = a.item_i0[it];
    const bool on = lane < a.item_i1[it] - i0;
    int32_t slot = 0;
    double x0 = 0, x1 = 0, x2 = 0;
    if (on) {
        const int64_t t = a.inc_tgt[i0 + lane];
        slot = a.inc_slot[i0 + lane];
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    // a pair closer than 1e-15 (r = 0 in particular) needs the target within that
    // distance of the leaf's box: only then does the wave take the checked loop
    const bool close = on && box_dist2(x0, x1, x2, a.bmin + 3 * c, a.bmax + 3 * c) <= 1e-30;
    const bool any_close = __ballot(close) != 0;
    // every lane runs the loops (lanes without a target use x = 0 and store nothing), so
    // the source records stay wave-uniform scalar loads
    const T *__restrict__ wts = static_cast<const T *>(a.wts);
    const int32_t s = a.start[c], n = a.count[c];
    const int K = a.K;
    const int ws = __builtin_amdgcn_readfirstlane(6 * K);
    for (int r0 = 0; r0 < K; r0 += KB) {
        T u[KB][3];
#pragma unroll
        for (int r = 0; r < KB; ++r) u[r][0] = u[r][1] = u[r][2] = T(0);
        const T *__restrict__ wr = wts + 6 * r0;
        if (K == KB) {
            if (any_close)
                near_leaf<T, true, KB, 6 * KB>(a.geo, wr, ws, s, n, x0, x1, x2, u);
            else
                near_leaf<T, false, KB, 6 * KB>(a.geo, wr, ws, s, n, x0, x1, x2, u);
        } else {
            if (any_close)
                near_leaf<T, true, KB, 0>(a.geo, wr, ws, s, n, x0, x1, x2, u);
            else
                near_leaf<T, false, KB, 0>(a.geo, wr, ws, s, n, x0, x1, x2, u);
        }
        if (on) {
            T *o = static_cast<T *>(a.part) + (int64_t(slot) * K + r0) * 3;
#pragma unroll
            for (int r = 0; r < KB; ++r) {
                o[3 * r] = u[r][0];
                o[3 * r + 1] = u[r][1];
                o[3 * r + 2] = u[r][2];
            }
        }
    }
}

// Regularized Stokeslet + stresslet pair (FP64, one right-hand side), R^2 = |d|^2 + eps^2:
//   u_i += f_i (|d|^2 + 2 eps^2)/R^3 + d_i [(d.f)/R^3 + (d.h)(d.nu)/R^5 + (eps^2/2)(h.nu)/R^5]
//          + h_i (eps^2/2)(d.nu)/R^5 + nu_i (eps^2/2)(d.h)/R^5
// (the kernels S^eps_ij f_j + T^eps_ijl h_j nu_l).  With eps > 0 every pair is finite and
// summed, the coincident one included; with eps = 0 R = 0 only there, and it is skipped.
__device__ inline void pair_reg(double x0, double x1, double x2, const double g[6], const double w[6], double e2,
                                double u[3]) {
    const double d0 = x0 - g[0], d1 = x1 - g[1], d2 = x2 - g[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double R2 = r2 + e2;
    double ri = rsqrt(R2);
    ri = R2 > 0.0 ? ri : 0.0;
    const double ri3 = ri * ri * ri;
    const double ri5 = ri3 * ri * ri;
    const double dn = d0 * g[3] + d1 * g[4] + d2 * g[5];
    const double df = d0 * w[0] + d1 * w[1] + d2 * w[2];
    const double dh = d0 * w[3] + d1 * w[4] + d2 * w[5];
    const double hn = w[3] * g[3] + w[4] * g[4] + w[5] * g[5];
    const double he = 0.5 * e2 * ri5;
    const double cs = (r2 + 2.0 * e2) * ri3;
    const double sd = df * ri3 + (dh * dn) * ri5 + he * hn;
    const double sh = he * dn, sn = he * dh;
    u[0] += w[0] * cs + d0 * sd + w[3] * sh + g[3] * sn;
    u[1] += w[1] * cs + d1 * sd + w[4] * sh + g[4] * sn;
    u[2] += w[2] * cs + d2 * sd + w[5] * sh + g[5] * sn;
}

// one wave per item as k_near, with the regularized pair: the leaf's records are walked
// with a uniform pointer, four sources per batch
__global__ __launch_bounds__(64) void k_near_reg(NearArgs a) {
    const int32_t it = xcd_item<XCD_CHUNK_NEAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int32_t c = a.item_leaf[it];
    const int32_t i0 = a.item_i0[it];
    const bool on = lane < a.item_i1[it] - i0;
    int32_t slot = 0;
    double x0 = 0, x1 = 0, x2 = 0;
    if (on) {
        const int64_t t = a.inc_tgt[i0 + lane];
        slot = a.inc_slot[i0 + lane];
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    const int32_t s = a.start[c], n = a.count[c];
    const STK_CONST_AS double *g = (const STK_CONST_AS double *)(a.geo) + 6 * int64_t(s);
    const STK_CONST_AS double *w = (const STK_CONST_AS double *)(a.wts) + 6 * int64_t(s);
    const double e2 = a.eps2;
    double u[3] = {0.0, 0.0, 0.0};
    int32_t left = n;
    for (; left >= 4; left -= 4, g += 24, w += 24) {
        double gb[4][6], wb[4][6];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                gb[b][q] = g[6 * b + q];
                wb[b][q] = w[6 * b + q];
            }
#pragma unroll
        for (int b = 0; b < 4; ++b) pair_reg(x0, x1, x2, gb[b], wb[b], e2, u);
    }
    for (; left > 0; --left, g += 6, w += 6) {
        double gc[6], wc[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            gc[q] = g[q];
            wc[q] = w[q];
        }
        pair_reg(x0, x1, x2, gc, wc, e2, u);
    }
    if (on) {
        double *o = static_cast<double *>(a.part) + int64_t(slot) * 3;
        o[0] = u[0];
        o[1] = u[1];
        o[2] = u[2];
    }
}

// Near field for K right-hand sides on the matrix cores (FP32 mixed precision).  With
// the pair written as u_i = sum_j K_ij w_j over w = (f, h):
//   K_ij = delta_ij / r + d_i d_j / r^3,   K_i(3+j) = d_i d_j (d.nu) / r^5,
// an item (one leaf against up to 64 targets, in four blocks of 16) is a product of the
// (target x source) kernel blocks with the (source x RHS) weights.  Per block of four
// sources, lane l forms the 3x6 block of the pair (target 16 tb + l % 16, source
// 4 yb + l / 16) and loads the six weights of (source 4 yb + l / 16, RHS r0 + l % 16);
// v_mfma_f32_16x16x4_f32 then adds A[t][y] B[y][r] over the four sources for each
// (i, j), so every lane supplies exactly the operand entries it computed (rows =
// targets, depth = the four sources, columns = 16 right-hand sides).  d and d.nu are
// FP64 as in the VALU kernel; the kernel entries and their sums are FP32.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool CHECK, bool TAIL>
__device__ inline void near_mfma_block(const double (&xt)[4][3], const double gy[6], const float wj[6], bool yv,
                                       f32x4 (&acc)[4][3]) {
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) {
        const double d0 = xt[tb][0] - gy[0], d1 = xt[tb][1] - gy[1], d2 = xt[tb][2] - gy[2];
        const double dn = d0 * gy[3] + d1 * gy[4] + d2 * gy[5];
        const float f[3] = {float(d0), float(d1), float(d2)};
        const float r2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
        float ri = __frsqrt_rn(r2);
        if constexpr (CHECK) ri = r2 > 0.0f ? ri : 0.0f;
        if constexpr (TAIL) ri = yv ? ri : 0.0f;  // padding source: a zero column (d is finite)
        const float r2i = ri * ri;
        const float a3 = ri * r2i;
        const float a5 = float(dn) * (a3 * r2i);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const float pij = f[i] * f[j];
                const float ks = i == j ? fmaf(pij, a3, ri) : pij * a3;
                acc[tb][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(ks, wj[j], acc[tb][i], 0, 0, 0);
                acc[tb][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(pij * a5, wj[3 + j], acc[tb][i], 0, 0, 0);
            }
        }
    }
}

template <bool CHECK>
__device__ inline void near_mfma_leaf(const double *__restrict__ geo, const float *__restrict__ wts, int K, int r,
                                      bool rv, int32_t s, int32_t n, int q4, const double (&xt)[4][3],
                                      f32x4 (&acc)[4][3]) {
    int32_t y0 = s;
    for (; y0 + 4 <= s + n; y0 += 4) {
        const int64_t y = y0 + q4;
        double gy[6];
        float wj[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            gy[q] = geo[6 * y + q];
            wj[q] = rv ? wts[(y * K + r) * 6 + q] : 0.0f;
        }
        near_mfma_block<CHECK, false>(xt, gy, wj, true, acc);
    }
    if (y0 < s + n) {  // last, partial block of four
        const int64_t y = y0 + q4;
        const bool yv = y < s + n;
        double gy[6] = {0, 0, 0, 0, 0, 0};
        float wj[6] = {0, 0, 0, 0, 0, 0};
        if (yv) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                gy[q] = geo[6 * y + q];
                wj[q] = rv ? wts[(y * K + r) * 6 + q] : 0.0f;
            }
        }
        near_mfma_block<CHECK, true>(xt, gy, wj, yv, acc);
    }
}

__global__ __launch_bounds__(64) void k_near_mfma(NearArgs a) {
    const int32_t it = xcd_item<XCD_CHUNK_NEAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int tl = lane & 15, q4 = lane >> 4;
    const int32_t c = a.item_leaf[it];
    const int32_t i0 = a.item_i0[it];
    const int32_t nt = a.item_i1[it] - i0;
    // this lane's A rows: targets 16 tb + tl of the item (rows past nt compute unused
    // values from x = 0 and are never stored)
    double xt[4][3];
    bool close = false;
#pragma unroll
    for (int tb = 0; tb < 4; ++tb) {
        xt[tb][0] = xt[tb][1] = xt[tb][2] = 0.0;
        if (16 * tb + tl < nt) {
            const int64_t t = a.inc_tgt[i0 + 16 * tb + tl];
            xt[tb][0] = a.tpos[3 * t];
            xt[tb][1] = a.tpos[3 * t + 1];
            xt[tb][2] = a.tpos[3 * t + 2];
            close = close || box_dist2(xt[tb][0], xt[tb][1], xt[tb][2], a.bmin + 3 * c, a.bmax + 3 * c) <= 1e-30;
        }
    }
    const bool any_close = __ballot(close) != 0;
    const float *__restrict__ wts = static_cast<const float *>(a.wts);
    const int32_t s = a.start[c], n = a.count[c];
    const int K = a.K;
    for (int r0 = 0; r0 < K; r0 += 16) {
        const int r = r0 + tl;
        const bool rv = r < K;
        f32x4 acc[4][3];
#pragma unroll
        for (int tb = 0; tb < 4; ++tb)
#pragma unroll
            for (int i = 0; i < 3; ++i) acc[tb][i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        if (any_close)
            near_mfma_leaf<true>(a.geo, wts, K, r, rv, s, n, q4, xt, acc);
        else
            near_mfma_leaf<false>(a.geo, wts, K, r, rv, s, n, q4, xt, acc);
        // lane holds rows 4 q4 + v (v = 0..3) of each target block, column tl
        if (rv) {
            float *part = static_cast<float *>(a.part);
#pragma unroll
            for (int tb = 0; tb < 4; ++tb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int idx = 16 * tb + 4 * q4 + v;
                    if (idx < nt) {
                        float *o = part + (int64_t(a.inc_slot[i0 + idx]) * K + r) * 3;
                        o[0] = acc[tb][0][v];
                        o[1] = acc[tb][1][v];
                        o[2] = acc[tb][2][v];
                    }
                }
        }
    }
}

// per (target, right-hand side): its partials in near-list order, compensated, to FP64
template <typename T>
__global__ void k_near_reduce(const T *__restrict__ part, const int32_t *__restrict__ toff, int64_t m, int K,
                              double *__restrict__ unear) {
    const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= m * K) return;
    const int64_t t = id / K;
    const int r = int(id - t * K);
    Comp<T> acc[3];
    for (int32_t k = toff[t]; k < toff[t + 1]; ++k) {
        const T *p = part + (int64_t(k) * K + r) * 3;
        acc[0].add(p[0]);
        acc[1].add(p[1]);
        acc[2].add(p[2]);
    }
    unear[3 * id] = acc[0].value();
    unear[3 * id + 1] = acc[1].value();
    unear[3 * id + 2] = acc[2].value();
}

template <typename T, int KB> void launch_near(const NearArgs &na, hipStream_t s) {
    if (na.nitems > 0) {
        hipLaunchKernelGGL((k_near<T, KB>), dim3(xcd_item_blocks<XCD_CHUNK_NEAR>(na.nitems)), dim3(64), 0, s, na);
        STK_CHECK_LAUNCH();
    }
}

}  // namespace

void cluster_major(Tree &t, ClusterMajor &cm, const int32_t *off, const int32_t *node, const uint64_t *mask,
                   int64_t ne, int32_t ng, int64_t m, int max_pc, const int32_t *tcount, hipStream_t s) {
    const CmInput in{off, node, mask, ne, ng, m, max_pc, tcount};
    cm_stage1(t, cm, in, s);
    cm_stage2(t, cm, in, s);
    cm_stage3(t, cm, in, s);
}

namespace {
int cm_key_bits(int32_t nn) {
    int bits = 1;
    while ((int64_t(1) << bits) <= int64_t(nn)) ++bits;
    return bits;
}
}  // namespace

// stage 1: the sort keys of the kept entries (node, entry); when few are kept (max_pc < 64)
// they are compacted first and their number is requested
void cm_stage1(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s) {
    const int32_t nn = int32_t(t.nnodes);
    const int64_t ne = in.ne;
    uint64_t *keys = reserve<uint64_t>(cm.keys, size_t(ne) + 1);
    int32_t *ent = reserve<int32_t>(cm.ent, size_t(ne) + 1);
    reserve<int32_t>(cm.pc, size_t(ne) + 1);
    reserve<int32_t>(cm.pos, size_t(ne) + 1);
    reserve<int32_t>(cm.incoff, size_t(ne) + 1);
    cm.nk = ne;
    cm.nk_pending = false;
    if (ne > 0 && in.max_pc < 64) {
        // few entries kept: compact them, then sort only those
        int32_t *flag = cm.pc.as<int32_t>();
        int32_t *fpos = cm.incoff.as<int32_t>();
        hipLaunchKernelGGL(k_cm_flag, dim3(nblk(ne, 256)), dim3(256), 0, s, in.mask, ne, in.max_pc, flag);
        STK_CHECK_LAUNCH();
        scan_exclusive_i32(flag, fpos, ne, cm.s_scan, s);
        hipLaunchKernelGGL(k_cm_compact, dim3(nblk(ne, 256)), dim3(256), 0, s, in.node, in.mask, ne, in.max_pc, fpos,
                           keys, ent);
        STK_CHECK_LAUNCH();
        const PeekSrc src{fpos + ne, 4};
        peek_start(cm.peek, s, 1, &src);
        cm.nk_pending = true;
    } else if (ne > 0) {
        hipLaunchKernelGGL(k_cm_keys, dim3(nblk(ne, 256)), dim3(256), 0, s, in.node, in.mask, ne, nn, in.max_pc, keys,
                           ent);
        STK_CHECK_LAUNCH();
    }
}

// stage 2: the sort, each sorted entry's incidences, per-target and per-node offsets; the
// totals are requested
void cm_stage2(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s) {
    const int32_t nn = int32_t(t.nnodes);
    const int64_t m = in.m;
    if (cm.nk_pending) {
        peek_wait(cm.peek, s, 1, &cm.nk);
        cm.nk_pending = false;
    }
    const int64_t nk = cm.nk;
    uint64_t *keys = cm.keys.as<uint64_t>();
    int32_t *ent = cm.ent.as<int32_t>();
    int32_t *pc = cm.pc.as<int32_t>();
    int32_t *pos = cm.pos.as<int32_t>();
    int32_t *incoff = cm.incoff.as<int32_t>();
    // kept entries sorted by node (stable: group order within a node), the others last
    radix_sort_pairs(cm.s_keys2, cm.s_vals2, cm.s_hist, keys, ent, nk, cm_key_bits(nn), s);
    if (nk > 0) {
        hipLaunchKernelGGL(k_cm_pos, dim3(nblk(nk, 256)), dim3(256), 0, s, ent, in.mask, nk, in.max_pc, pc, pos);
        STK_CHECK_LAUNCH();
    }
    scan_exclusive_i32(pc, incoff, nk, cm.s_scan, s);
    // per target: first slot (exclusive scan of its kept-entry count, sorted order)
    const int32_t *tcount = in.tcount;
    if (!tcount) {
        int32_t *tc = reserve<int32_t>(cm.tcnt, size_t(m) + 1);
        if (in.ng > 0) {
            hipLaunchKernelGGL(k_cm_tcount, dim3(in.ng), dim3(64), 0, s, in.off, in.mask, m, in.max_pc, tc);
            STK_CHECK_LAUNCH();
        }
        tcount = tc;
    }
    int32_t *toff = reserve<int32_t>(cm.toff, size_t(m) + 1);
    scan_exclusive_i32(tcount, toff, m, cm.s_scan, s);
    // per node: entry range, incidence range, items of up to 64 incidences
    int32_t *eoff = reserve<int32_t>(cm.eoff, size_t(nn) + 1);
    int32_t *loff = reserve<int32_t>(cm.loff, size_t(nn) + 1);
    int32_t *icnt = reserve<int32_t>(cm.icnt, size_t(nn) + 1);
    int32_t *ioff = reserve<int32_t>(cm.ioff, size_t(nn) + 1);
    hipLaunchKernelGGL(k_cm_nodes, dim3(nblk(int64_t(nn) + 1, 256)), dim3(256), 0, s, keys, nk, nn, incoff, 64, eoff,
                       loff, icnt);
    STK_CHECK_LAUNCH();
    scan_exclusive_i32(icnt, ioff, nn, cm.s_scan, s);
    const PeekSrc src[3] = {{incoff + nk, 4}, {ioff + nn, 4}, {toff + m, 4}};
    peek_start(cm.peek, s, 3, src);
}

// stage 3: the totals; the incidence and item arrays
void cm_stage3(Tree &t, ClusterMajor &cm, const CmInput &in, hipStream_t s) {
    const int32_t nn = int32_t(t.nnodes);
    int64_t tot[3];
    peek_wait(cm.peek, s, 3, tot);
    if (tot[0] != tot[2]) throw Error(STK_EDEVICE, "lists: incidence count differs from the per-target counts");
    cm.n_inc = tot[0];
    cm.n_items = int32_t(tot[1]);
    int32_t *inc_tgt = reserve<int32_t>(cm.inc_tgt, size_t(cm.n_inc) + 1);
    int32_t *inc_slot = reserve<int32_t>(cm.inc_slot, size_t(cm.n_inc) + 1);
    int32_t *inode = reserve<int32_t>(cm.item_node, size_t(cm.n_items) + 1);
    int32_t *i0 = reserve<int32_t>(cm.item_i0, size_t(cm.n_items) + 1);
    int32_t *i1 = reserve<int32_t>(cm.item_i1, size_t(cm.n_items) + 1);
    if (cm.n_items > 0) {
        hipLaunchKernelGGL(k_item_fill, dim3(nblk(cm.n_items, 256)), dim3(256), 0, s, cm.loff.as<int32_t>(),
                           cm.ioff.as<int32_t>(), nn, 64, cm.n_items, inode, i0, i1);
        STK_CHECK_LAUNCH();
    }
    if (in.ng > 0) {
        hipLaunchKernelGGL(k_cm_fill, dim3(in.ng), dim3(64), 0, s, in.off, in.mask, in.max_pc, cm.pos.as<int32_t>(),
                           cm.incoff.as<int32_t>(), cm.toff.as<int32_t>(), in.m, inc_tgt, inc_slot);
        STK_CHECK_LAUNCH();
    }
}

void near_field(Tree &t, Plan &pl, double *unear, hipStream_t s, bool reduce) {
    cluster_major(t, pl.ncm, pl.near_off.as<int32_t>(), pl.near_node.as<int32_t>(), pl.near_mask.as<uint64_t>(),
                  pl.n_near_entries, pl.ngroups, pl.m, 64, pl.cnt_near.as<int32_t>(), s);
    prof_mark(STK_PHASE_LISTS, s);
    near_kernels(t, pl, unear, s, reduce);
}

void near_kernels(Tree &t, Plan &pl, double *unear, hipStream_t s, bool reduce) {
    const int64_t m = pl.m;
    ClusterMajor &cm = pl.ncm;
    // source records computed beside the lists (on another stream) must be complete from
    // here on
    if (pl.records_ready) {
        STK_HIP(hipStreamWaitEvent(s, pl.records_ready, 0));
        pl.records_ready = nullptr;
    }
    const int32_t *ileaf = cm.item_node.as<int32_t>(), *i0 = cm.item_i0.as<int32_t>(), *i1 = cm.item_i1.as<int32_t>();
    const int32_t *inc_tgt = cm.inc_tgt.as<int32_t>(), *inc_slot = cm.inc_slot.as<int32_t>();
    const int32_t *toff = cm.toff.as<int32_t>();

    const int K = t.k_rhs;
    const size_t tsz = t.prec == STK_FP64 ? sizeof(double) : sizeof(float);
    void *part = reserve<unsigned char>(cm.part, tsz * 3 * size_t(cm.n_inc) * K + tsz);
    NearArgs na{pl.tpos_p, ileaf, i0, i1, inc_tgt, inc_slot, t.nstart.as<int32_t>(),
                t.ncount.as<int32_t>(), t.nbmin.as<double>(), t.nbmax.as<double>(), t.geo.as<double>(), t.wts.p,
                part, cm.n_items, K};
    const int64_t mk = m * K;
    if (pl.reg_eps >= 0.0) {
        if (t.prec != STK_FP64 || K != 1) throw Error(STK_EINVAL, "regularized kernels: FP64, one right-hand side");
        na.eps2 = pl.reg_eps * pl.reg_eps;
        if (na.nitems > 0) {
            hipLaunchKernelGGL(k_near_reg, dim3(xcd_item_blocks<XCD_CHUNK_NEAR>(na.nitems)), dim3(64), 0, s, na);
            STK_CHECK_LAUNCH();
        }
        if (reduce && mk > 0) {
            hipLaunchKernelGGL(k_near_reduce<double>, dim3(nblk(mk, 256)), dim3(256), 0, s,
                               static_cast<const double *>(part), toff, m, K, unear);
            STK_CHECK_LAUNCH();
        }
    } else if (t.prec == STK_FP64) {
        launch_near<double, 1>(na, s);
        if (reduce && mk > 0) {
            hipLaunchKernelGGL(k_near_reduce<double>, dim3(nblk(mk, 256)), dim3(256), 0, s,
                               static_cast<const double *>(part), toff, m, K, unear);
            STK_CHECK_LAUNCH();
        }
    } else {
        if (pl.tiles.near_mfma) {
            if (na.nitems > 0) {
                hipLaunchKernelGGL(k_near_mfma, dim3(xcd_item_blocks<XCD_CHUNK_NEAR>(na.nitems)), dim3(64), 0, s, na);
                STK_CHECK_LAUNCH();
            }
        } else if (pl.tiles.near_kb == 4)
            launch_near<float, 4>(na, s);
        else if (pl.tiles.near_kb == 2)
            launch_near<float, 2>(na, s);
        else
            launch_near<float, 1>(na, s);
        if (reduce && mk > 0) {
            hipLaunchKernelGGL(k_near_reduce<float>, dim3(nblk(mk, 256)), dim3(256), 0, s,
                               static_cast<const float *>(part), toff, m, K, unear);
            STK_CHECK_LAUNCH();
        }
    }
    prof_mark(STK_PHASE_NEAR, s);
}

}  // namespace stk
