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
// which is f_i/r + d_i (d.f)/r^3 + d_i (d.h)(d.nu)/r^5, in two FMAs per component.
// g = (y, nu) and w = (f, h) are wave-uniform (held in SGPRs).  CHECK: a pair with
// r = 0 may occur (the coincident source is skipped, Sec. 2); without it the caller
// has shown that every pair of the leaf is at distance > 1e-15.
template <bool CHECK>
__device__ inline void pair_f64(double x0, double x1, double x2, const double g[6], const double w[6], double &u0,
                                double &u1, double &u2) {
    const double d0 = x0 - g[0], d1 = x1 - g[1], d2 = x2 - g[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    double ri = rsqrt(r2);
    if constexpr (CHECK) ri = r2 > 0.0 ? ri : 0.0;
    const double r2i = ri * ri;
    const double dn = d0 * g[3] + d1 * g[4] + d2 * g[5];
    const double df = d0 * w[0] + d1 * w[1] + d2 * w[2];
    const double dh = d0 * w[3] + d1 * w[4] + d2 * w[5];
    const double sc = fma(dh, dn * r2i, df) * r2i;
    u0 = fma(ri, fma(d0, sc, w[0]), u0);
    u1 = fma(ri, fma(d1, sc, w[1]), u1);
    u2 = fma(ri, fma(d2, sc, w[2]), u2);
}

// Mixed precision: d = x - y and d.nu in FP64 (on a surface with nu the normal d.nu is
// O(|d|^2), so its absolute rounding must stay at FP64 level), the rest in FP32.
template <bool CHECK>
__device__ inline void pair_mixed(double x0, double x1, double x2, const double g[6], const float w[6], float &u0,
                                  float &u1, float &u2) {
    const double d0 = x0 - g[0], d1 = x1 - g[1], d2 = x2 - g[2];
    const double dn = d0 * g[3] + d1 * g[4] + d2 * g[5];
    const float f0 = float(d0), f1 = float(d1), f2 = float(d2);
    const float r2 = f0 * f0 + f1 * f1 + f2 * f2;
    float ri = __frsqrt_rn(r2);
    if constexpr (CHECK) ri = r2 > 0.0f ? ri : 0.0f;
    const float r2i = ri * ri;
    const float df = f0 * w[0] + f1 * w[1] + f2 * w[2];
    const float dh = f0 * w[3] + f1 * w[4] + f2 * w[5];
    const float sc = fmaf(dh, float(dn) * r2i, df) * r2i;
    u0 = fmaf(ri, fmaf(f0, sc, w[0]), u0);
    u1 = fmaf(ri, fmaf(f1, sc, w[1]), u1);
    u2 = fmaf(ri, fmaf(f2, sc, w[2]), u2);
}

// sum over sources [s, s + n) of one leaf; records are read four at a time (one wait on
// the scalar cache per batch of four)
template <typename T, bool CHECK>
__device__ inline void near_leaf(const double *__restrict__ geo, const T *__restrict__ wts, int32_t s, int32_t n,
                                 double x0, double x1, double x2, T &u0, T &u1, T &u2) {
    int32_t j = s;
    for (; j + 4 <= s + n; j += 4) {
        double gb[4][6];
        T wb[4][6];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                gb[b][q] = geo[6 * int64_t(j + b) + q];
                wb[b][q] = wts[6 * int64_t(j + b) + q];
            }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if constexpr (sizeof(T) == 8)
                pair_f64<CHECK>(x0, x1, x2, gb[b], reinterpret_cast<const double *>(wb[b]), u0, u1, u2);
            else
                pair_mixed<CHECK>(x0, x1, x2, gb[b], reinterpret_cast<const float *>(wb[b]), u0, u1, u2);
        }
    }
    for (; j < s + n; ++j) {
        double gc[6];
        T wc[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            gc[q] = geo[6 * int64_t(j) + q];
            wc[q] = wts[6 * int64_t(j) + q];
        }
        if constexpr (sizeof(T) == 8)
            pair_f64<CHECK>(x0, x1, x2, gc, reinterpret_cast<const double *>(wc), u0, u1, u2);
        else
            pair_mixed<CHECK>(x0, x1, x2, gc, reinterpret_cast<const float *>(wc), u0, u1, u2);
    }
}

// squared distance from x to the closed box [lo, hi] (FP64)
__device__ inline double box_dist2(double x0, double x1, double x2, const double *lo, const double *hi) {
    const double e0 = fmax(fmax(lo[0] - x0, x0 - hi[0]), 0.0);
    const double e1 = fmax(fmax(lo[1] - x1, x1 - hi[1]), 0.0);
    const double e2 = fmax(fmax(lo[2] - x2, x2 - hi[2]), 0.0);
    return e0 * e0 + e1 * e1 + e2 * e2;
}

// ---- leaf-major plan -------------------------------------------------------------------
// sorted entry k: popcount of its mask; pos[e] = sorted position of entry e
__global__ void k_nl_pos(const int32_t *__restrict__ ent, const uint64_t *__restrict__ mask, int64_t ne,
                         int32_t *__restrict__ pc, int32_t *__restrict__ pos) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= ne) return;
    const int32_t e = ent[k];
    pc[k] = __popcll(mask[e]);
    pos[e] = int32_t(k);
}

// loff[c] = first incidence of leaf c, c in [0, nn]
__global__ void k_nl_loff(const int32_t *__restrict__ eoff, const int32_t *__restrict__ incoff, int32_t nn,
                          int32_t *__restrict__ loff) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nn) return;
    loff[c] = incoff[eoff[c]];
}

// one wave per group: lane l walks the group's entries in list order and places each of
// its incidences (target, slot) at the incidence's leaf-major position
__global__ __launch_bounds__(64) void k_nl_fill(const int32_t *__restrict__ off, const uint64_t *__restrict__ mask,
                                                const int32_t *__restrict__ pos, const int32_t *__restrict__ incoff,
                                                const int32_t *__restrict__ toff, int64_t m,
                                                int32_t *__restrict__ inc_tgt, int32_t *__restrict__ inc_slot) {
    const int32_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t t = int64_t(g) * 64 + lane;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t slot = t < m ? toff[t] : 0;
    for (int32_t e = off[g]; e < off[g + 1]; ++e) {
        const uint64_t mk = mask[e];
        if ((mk >> lane) & 1ull) {
            const int32_t q = incoff[pos[e]] + __popcll(mk & lt);
            inc_tgt[q] = int32_t(t);
            inc_slot[q] = slot++;
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
    const void *wts;                       // (n,6) f, h in T
    void *part;                            // (incidences, 3) T
    int32_t nitems;
};

// one wave per item: the item's leaf against up to 64 of its targets.  Items of one leaf
// are consecutive and go to one XCD, so the leaf's records are shared in its L2.
template <typename T> __global__ __launch_bounds__(64) void k_near(NearArgs a) {
    const int32_t it = xcd_group(a.nitems);
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
    if (on) {
        const T *__restrict__ wts = static_cast<const T *>(a.wts);
        const int32_t s = a.start[c], n = a.count[c];
        T u0 = T(0), u1 = T(0), u2 = T(0);
        if (any_close)
            near_leaf<T, true>(a.geo, wts, s, n, x0, x1, x2, u0, u1, u2);
        else
            near_leaf<T, false>(a.geo, wts, s, n, x0, x1, x2, u0, u1, u2);
        T *o = static_cast<T *>(a.part) + 3 * int64_t(slot);
        o[0] = u0;
        o[1] = u1;
        o[2] = u2;
    }
}

// per target: its partials in near-list order, compensated, to FP64
template <typename T>
__global__ void k_near_reduce(const T *__restrict__ part, const int32_t *__restrict__ toff, int64_t m,
                              double *__restrict__ unear) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= m) return;
    Comp<T> acc[3];
    for (int32_t k = toff[t]; k < toff[t + 1]; ++k) {
        acc[0].add(part[3 * int64_t(k)]);
        acc[1].add(part[3 * int64_t(k) + 1]);
        acc[2].add(part[3 * int64_t(k) + 2]);
    }
    unear[3 * t] = acc[0].value();
    unear[3 * t + 1] = acc[1].value();
    unear[3 * t + 2] = acc[2].value();
}

}  // namespace

void near_field(Tree &t, Plan &pl, double *unear, hipStream_t s) {
    const int64_t m = pl.m;
    const int64_t ne = pl.n_near_entries;
    const int32_t nn = int32_t(t.nnodes);
    const int32_t ng = pl.ngroups;
    const int32_t *off = pl.near_off.as<int32_t>();
    const int32_t *node = pl.near_node.as<int32_t>();
    const uint64_t *mask = pl.near_mask.as<uint64_t>();

    // entries sorted by leaf (stable: group order within a leaf)
    uint64_t *keys = reserve<uint64_t>(pl.nl_keys, size_t(ne) + 1);
    int32_t *ent = reserve<int32_t>(pl.nl_ent, size_t(ne) + 1);
    if (ne > 0) {
        hipLaunchKernelGGL(k_node_keys, dim3(nblk(ne, 256)), dim3(256), 0, s, node, ne, keys, ent);
        STK_CHECK_LAUNCH();
        int bits = 1;
        while ((int64_t(1) << bits) <= int64_t(nn)) ++bits;
        radix_sort_pairs(t, keys, ent, ne, bits, s);
    }
    int32_t *pc = reserve<int32_t>(pl.nl_pc, size_t(ne) + 1);
    int32_t *pos = reserve<int32_t>(pl.nl_pos, size_t(ne) + 1);
    int32_t *incoff = reserve<int32_t>(pl.nl_incoff, size_t(ne) + 1);
    if (ne > 0) {
        hipLaunchKernelGGL(k_nl_pos, dim3(nblk(ne, 256)), dim3(256), 0, s, ent, mask, ne, pc, pos);
        STK_CHECK_LAUNCH();
    }
    scan_exclusive_i32(pc, incoff, ne, t.s_scan, s);
    // per target: first slot (exclusive scan of the near-leaf counts, sorted order)
    int32_t *toff = reserve<int32_t>(pl.near_toff, size_t(m) + 1);
    scan_exclusive_i32(pl.cnt_near.as<int32_t>(), toff, m, t.s_scan, s);
    // per leaf: entry range, incidence range, items of up to 64 incidences
    int32_t *eoff = reserve<int32_t>(pl.nl_eoff, size_t(nn) + 1);
    int32_t *loff = reserve<int32_t>(pl.nl_loff, size_t(nn) + 1);
    int32_t *icnt = reserve<int32_t>(pl.nl_icnt, size_t(nn) + 1);
    int32_t *ioff = reserve<int32_t>(pl.nl_ioff, size_t(nn) + 1);
    hipLaunchKernelGGL(k_node_off, dim3(nblk(int64_t(nn) + 1, 256)), dim3(256), 0, s, keys, ne, nn, eoff);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_nl_loff, dim3(nblk(int64_t(nn) + 1, 256)), dim3(256), 0, s, eoff, incoff, nn, loff);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_item_count, dim3(nblk(nn, 256)), dim3(256), 0, s, loff, nn, 64, icnt);
    STK_CHECK_LAUNCH();
    scan_exclusive_i32(icnt, ioff, nn, t.s_scan, s);
    int32_t tot[3];
    STK_HIP(hipMemcpyAsync(&tot[0], incoff + ne, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    STK_HIP(hipMemcpyAsync(&tot[1], ioff + nn, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    STK_HIP(hipMemcpyAsync(&tot[2], toff + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    STK_HIP(hipStreamSynchronize(s));
    if (tot[0] != tot[2]) throw Error(STK_EDEVICE, "near lists: incidence count differs from the per-target counts");
    pl.n_inc = tot[0];
    pl.n_near_items = tot[1];
    int32_t *inc_tgt = reserve<int32_t>(pl.inc_tgt, size_t(pl.n_inc) + 1);
    int32_t *inc_slot = reserve<int32_t>(pl.inc_slot, size_t(pl.n_inc) + 1);
    int32_t *ileaf = reserve<int32_t>(pl.item_leaf, size_t(pl.n_near_items) + 1);
    int32_t *i0 = reserve<int32_t>(pl.item_i0, size_t(pl.n_near_items) + 1);
    int32_t *i1 = reserve<int32_t>(pl.item_i1, size_t(pl.n_near_items) + 1);
    hipLaunchKernelGGL(k_item_fill, dim3(nblk(nn, 256)), dim3(256), 0, s, loff, ioff, nn, 64, ileaf, i0, i1);
    STK_CHECK_LAUNCH();
    if (ng > 0) {
        hipLaunchKernelGGL(k_nl_fill, dim3(ng), dim3(64), 0, s, off, mask, pos, incoff, toff, m, inc_tgt, inc_slot);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_LISTS, s);

    const size_t tsz = t.prec == STK_FP64 ? sizeof(double) : sizeof(float);
    void *part = reserve<unsigned char>(pl.near_part, tsz * 3 * size_t(pl.n_inc) + tsz);
    NearArgs na{pl.tpos.as<double>(), ileaf, i0, i1, inc_tgt, inc_slot, t.nstart.as<int32_t>(),
                t.ncount.as<int32_t>(), t.nbmin.as<double>(), t.nbmax.as<double>(), t.geo.as<double>(), t.wts.p,
                part, pl.n_near_items};
    if (t.prec == STK_FP64) {
        if (na.nitems > 0) {
            hipLaunchKernelGGL(k_near<double>, dim3(xcd_blocks(na.nitems)), dim3(64), 0, s, na);
            STK_CHECK_LAUNCH();
        }
        if (m > 0) {
            hipLaunchKernelGGL(k_near_reduce<double>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const double *>(part), toff, m, unear);
            STK_CHECK_LAUNCH();
        }
    } else {
        if (na.nitems > 0) {
            hipLaunchKernelGGL(k_near<float>, dim3(xcd_blocks(na.nitems)), dim3(64), 0, s, na);
            STK_CHECK_LAUNCH();
        }
        if (m > 0) {
            hipLaunchKernelGGL(k_near_reduce<float>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const float *>(part), toff, m, unear);
            STK_CHECK_LAUNCH();
        }
    }
    prof_mark(STK_PHASE_NEAR, s);
}

}  // namespace stk
