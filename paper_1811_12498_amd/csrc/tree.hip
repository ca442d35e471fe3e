// Octree over the sources (Sec. 5): root cube, Morton keys, radix sort, level-by-level
// subdivision, tight boxes, centres and radii.
//
// Geometry is exact: bounds are min/max reductions, centres 0.5 * (min + max), and the
// radius sqrt of the largest |y - y_c|^2, evaluated without contraction into FMA so
// every value is the correctly rounded result of the expression as written.
#include "stk_internal.hpp"
#include "stk_math.hpp"

#include <algorithm>
#include <cmath>

namespace stk {
namespace {

constexpr int BT = 256;

__device__ inline double atomic_max_nonneg(double *addr, double v) {
    // non-negative doubles order like their bit patterns
    return __longlong_as_double(
        (long long)atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v)));
}

// ---- bounds of the source set -----------------------------------------------------
__global__ __launch_bounds__(BT) void k_bounds(const double *__restrict__ src, int64_t n, double *__restrict__ part) {
    __shared__ double red[6][BT];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = int64_t(blockIdx.x) * BT + threadIdx.x; i < n; i += int64_t(gridDim.x) * BT)
        for (int a = 0; a < 3; ++a) {
            const double v = src[3 * i + a];
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + o]);
                red[3 + a][threadIdx.x] = fmax(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(BT) void k_bounds_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double red[6][BT];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += BT)
        for (int a = 0; a < 6; ++a) v[a] = a < 3 ? fmin(v[a], part[b * 6 + a]) : fmax(v[a], part[b * 6 + a]);
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int a = 0; a < 6; ++a)
                red[a][threadIdx.x] = a < 3 ? fmin(red[a][threadIdx.x], red[a][threadIdx.x + o])
                                            : fmax(red[a][threadIdx.x], red[a][threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---- Morton keys --------------------------------------------------------------------
__device__ inline uint64_t spread3(uint64_t v) {  // 21 bits -> every third bit
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

__global__ void k_keys(const double *__restrict__ pts, int64_t n, double lx, double ly, double lz, double scale,
                       int degenerate, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t key = 0;
    if (!degenerate) {
        const uint64_t qx = quant(pts[3 * i], lx, scale);
        const uint64_t qy = quant(pts[3 * i + 1], ly, scale);
        const uint64_t qz = quant(pts[3 * i + 2], lz, scale);
        key = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    }
    keys[i] = key;
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

// ---- subdivision -----------------------------------------------------------------------
// the root: every point, no children yet
__global__ void k_root(int32_t n, int32_t *__restrict__ level, int32_t *__restrict__ parent,
                       int32_t *__restrict__ child0, int32_t *__restrict__ nchild, int32_t *__restrict__ start,
                       int32_t *__restrict__ count) {
    if (threadIdx.x == 0) {
        level[0] = 0;
        parent[0] = -1;
        child0[0] = -1;
        nchild[0] = 0;
        start[0] = 0;
        count[0] = n;
    }
}

// The octant split of one node [s, s + c) by one wavefront (every lane calls it): the
// boundaries b_d = first index whose 3-bit digit at `shift` is >= d, d = 1..7 (the node's
// keys are sorted and share the bits above the digit, so the digits rise along the node).
// The seven searches run together: lanes 9(d-1) .. 9(d-1)+8 probe nine points of the
// interval still holding b_d, which shrinks about tenfold per round.  Lanes 0..8 write
// bnd9[d] = b_d (b_0 = s, b_8 = s + c); returns the number of non-empty octants.
__device__ inline int32_t split_node(const uint64_t *__restrict__ keys, int32_t s, int32_t c, int shift,
                                     int32_t *bnd9) {
    const int lane = threadIdx.x & 63;
    const int g = lane / 9, k = lane - 9 * g;  // boundary d = g + 1; lane 63 (g = 7) idles
    int32_t lo = s, hi = g < 7 ? s + c : s;    // b_d lies in [lo, hi]
    while (__ballot(lo < hi) != 0) {
        const int32_t len = hi - lo;
        const int np = len > 9 ? 9 : len;
        // probes: lo + (k + 1) len / 10 for an interval of ten or more, else every point
        const int32_t pos = len > 9 ? lo + int32_t(int64_t(k + 1) * len / 10) : lo + k;
        const bool ge = len > 0 && k < np && int((keys[pos] >> shift) & 7) >= g + 1;
        const uint64_t bal = __ballot(ge);
        if (len > 0) {
            const uint32_t gb = uint32_t(bal >> (9 * g)) & 0x1ffu;
            const int j = gb ? __builtin_ctz(gb) : np;  // probes below the boundary
            if (len <= 9) {
                lo = hi = lo + j;
            } else {
                const int32_t nlo = j > 0 ? lo + int32_t(int64_t(j) * len / 10) + 1 : lo;
                hi = j < 9 ? lo + int32_t(int64_t(j + 1) * len / 10) : hi;
                lo = nlo;
            }
        }
    }
    const int32_t bd = __shfl(lo, lane >= 1 && lane <= 7 ? 9 * (lane - 1) : 0, 64);
    const int32_t b = lane == 0 ? s : (lane == 8 ? s + c : bd);
    if (lane < 9) bnd9[lane] = b;
    const int32_t next = __shfl(b, lane < 63 ? lane + 1 : 63, 64);
    return int32_t(__popcll(__ballot(lane < 8 && next > b)));
}

// Node `node` (at level lev) gets its k children, the first at index c, one per non-empty
// octant of bnd9.  cs / cc, if given, also receive each child's (start, count) at its
// index relative to c0.
__device__ inline void emit_node(int32_t node, int32_t k, int32_t c, int32_t c0, const int32_t *bnd9, int32_t lev,
                                 int32_t *__restrict__ level, int32_t *__restrict__ parent,
                                 int32_t *__restrict__ child0, int32_t *__restrict__ nchild,
                                 int32_t *__restrict__ start, int32_t *__restrict__ count, int32_t *cs, int32_t *cc) {
    if (k == 0) {
        child0[node] = -1;
        nchild[node] = 0;
        return;
    }
    child0[node] = c;
    nchild[node] = k;
    for (int d = 0; d < 8; ++d) {
        const int32_t b = bnd9[d], e = bnd9[d + 1];
        if (e > b) {
            level[c] = lev + 1;
            parent[c] = node;
            child0[c] = -1;
            nchild[c] = 0;
            start[c] = b;
            count[c] = e - b;
            if (cs) {
                cs[c - c0] = b;
                cc[c - c0] = e - b;
            }
            ++c;
        }
    }
}

// One wavefront per node of the level: nodes with more than n0 points are split
// (bnd[9 i ..] their octant bounds), nch[i] = number of children.
__global__ __launch_bounds__(BT) void k_split_count(const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ start,
                                                    const int32_t *__restrict__ count, int32_t lb, int32_t nlev,
                                                    int shift, int32_t n0, int32_t *__restrict__ nch,
                                                    int32_t *__restrict__ bnd) {
    const int32_t i = int32_t((int64_t(blockIdx.x) * BT + threadIdx.x) >> 6);  // uniform per wave
    const int lane = threadIdx.x & 63;
    if (i >= nlev) return;
    const int32_t s = start[lb + i], c = count[lb + i];
    const int32_t k = c > n0 ? split_node(keys, s, c, shift, bnd + 9 * i) : 0;
    if (lane == 0) nch[i] = k;
}

__global__ void k_split_emit(int32_t lb, int32_t nlev, int32_t le, int32_t lev, const int32_t *__restrict__ nch,
                             const int32_t *__restrict__ choff, const int32_t *__restrict__ bnd,
                             int32_t *__restrict__ level, int32_t *__restrict__ parent, int32_t *__restrict__ child0,
                             int32_t *__restrict__ nchild, int32_t *__restrict__ start, int32_t *__restrict__ count) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlev) return;
    emit_node(lb + i, nch[i], le + choff[i], 0, bnd + 9 * i, lev, level, parent, child0, nchild, start, count,
              nullptr, nullptr);
}

// The levels of at most TOP_NODES nodes from the root down, in one block: its waves split
// a level's nodes, wave 0 scans the child counts, its threads emit the children, and the
// next level's (start, count) stay in LDS.  out (the host's pinned slots): out[0] = levels
// done, out[1] = the level reached, out[2] / out[3] = its first node / one past its last,
// out[4] = 1 if no node of the last level done split (the tree is complete), out[5 + j] =
// the first node of level j + 1 for each level j done.
constexpr int TOP_T = 1024;
constexpr int TOP_NODES = 128;

__global__ __launch_bounds__(TOP_T) void k_split_top(const uint64_t *__restrict__ keys, int32_t n, int32_t n0,
                                                     int32_t *__restrict__ level, int32_t *__restrict__ parent,
                                                     int32_t *__restrict__ child0, int32_t *__restrict__ nchild,
                                                     int32_t *__restrict__ start, int32_t *__restrict__ count,
                                                     int64_t *__restrict__ out) {
    __shared__ int32_t cs[8 * TOP_NODES], cc[8 * TOP_NODES];  // the level's nodes: start, count
    __shared__ int32_t nch[TOP_NODES], choff[TOP_NODES + 1], bnd[9 * TOP_NODES];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        cs[0] = 0;
        cc[0] = n;
    }
    __syncthreads();
    int32_t lb = 0, le = 1, lev = 0, done = 0, nlv = 0;  // the same in every thread
    while (lev < STK_MAX_LEVEL && le - lb <= TOP_NODES) {
        const int32_t nlev = le - lb;
        for (int32_t i = wave; i < nlev; i += TOP_T / 64) {
            const int32_t c = cc[i];
            const int32_t k = c > n0 ? split_node(keys, cs[i], c, 3 * (STK_MAX_LEVEL - 1 - lev), bnd + 9 * i) : 0;
            if (lane == 0) nch[i] = k;
        }
        __syncthreads();
        if (wave == 0) {  // exclusive scan of nch[0, nlev), two per lane
            static_assert(TOP_NODES <= 128, "two counts per lane of one wave");
            const int32_t a0 = 2 * lane < nlev ? nch[2 * lane] : 0;
            const int32_t a1 = 2 * lane + 1 < nlev ? nch[2 * lane + 1] : 0;
            int32_t x = a0 + a1;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            const int32_t ex = x - a0 - a1;
            if (2 * lane < nlev) choff[2 * lane] = ex;
            if (2 * lane + 1 < nlev) choff[2 * lane + 1] = ex + a0;
            if (lane == 63) choff[TOP_NODES] = x;
        }
        __syncthreads();
        const int32_t total = choff[TOP_NODES];
        if (tid < nlev)
            emit_node(lb + tid, nch[tid], le + choff[tid], le, bnd + 9 * tid, lev, level, parent, child0, nchild,
                      start, count, cs, cc);
        __syncthreads();
        if (tid == 0) out[5 + nlv] = le;
        ++nlv;
        if (total == 0) {
            done = 1;
            break;
        }
        lb = le;
        le += total;
        ++lev;
    }
    if (tid == 0) {
        out[0] = nlv;
        out[1] = lev;
        out[2] = lb;
        out[3] = le;
        out[4] = done;
    }
}

// ---- boxes ----------------------------------------------------------------------------
__global__ __launch_bounds__(BT) void k_leaf_box(const double *__restrict__ pos, const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ count,
                                                 const int32_t *__restrict__ nchild, double *__restrict__ bmin,
                                                 double *__restrict__ bmax, double *__restrict__ center) {
    const int32_t node = blockIdx.x;
    if (nchild[node] != 0) return;
    __shared__ double red[6][BT];
    const int32_t s = start[node], c = count[node];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = threadIdx.x; i < c; i += BT)
        for (int a = 0; a < 3; ++a) {
            const double v = pos[3 * int64_t(s + i) + a];
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = lo[a];
        red[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fmin(red[a][threadIdx.x], red[a][threadIdx.x + o]);
                red[3 + a][threadIdx.x] = fmax(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        const double l = red[a][0], h = red[3 + a][0];
        bmin[3 * node + a] = l;
        bmax[3 * node + a] = h;
        center[3 * node + a] = 0.5 * (l + h);
    }
}

// an inner node's box: the union of its children's, centre its midpoint
__device__ inline void inner_box(int32_t node, const int32_t *__restrict__ child0, const int32_t *__restrict__ nchild,
                                 double *__restrict__ bmin, double *__restrict__ bmax, double *__restrict__ center) {
    const int32_t k = nchild[node];
    if (k == 0) return;
    const int32_t c0 = child0[node];
    for (int a = 0; a < 3; ++a) {
        double l = bmin[3 * c0 + a], h = bmax[3 * c0 + a];
        for (int32_t c = 1; c < k; ++c) {
            l = fmin(l, bmin[3 * (c0 + c) + a]);
            h = fmax(h, bmax[3 * (c0 + c) + a]);
        }
        bmin[3 * node + a] = l;
        bmax[3 * node + a] = h;
        center[3 * node + a] = 0.5 * (l + h);
    }
}

__global__ void k_inner_box(int32_t lb, int32_t nlev, const int32_t *__restrict__ child0,
                            const int32_t *__restrict__ nchild, double *__restrict__ bmin, double *__restrict__ bmax,
                            double *__restrict__ center) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlev) inner_box(lb + i, child0, nchild, bmin, bmax, center);
}

// the boxes of levels top, top - 1, .., 0 (each of at most TOP_BOX_NODES nodes) by one
// block, level by level: a level's boxes are read by the next only after the barrier
constexpr int TOP_BOX_NODES = 4096;
struct LevelBegins {
    int32_t b[STK_MAX_LEVEL + 2];
};
__global__ __launch_bounds__(1024) void k_inner_box_top(int32_t top, LevelBegins lv, const int32_t *__restrict__ child0,
                                                        const int32_t *__restrict__ nchild, double *__restrict__ bmin,
                                                        double *__restrict__ bmax, double *__restrict__ center) {
    for (int32_t l = top; l >= 0; --l) {
        for (int32_t node = lv.b[l] + int32_t(threadIdx.x); node < lv.b[l + 1]; node += 1024)
            inner_box(node, child0, nchild, bmin, bmax, center);
        __syncthreads();
    }
}

// ---- radii over (node, chunk) work items ---------------------------------------------
__global__ void k_chunk_count(const int32_t *__restrict__ count, int32_t nn, int32_t *__restrict__ out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nn) out[i] = (count[i] + CHUNK - 1) / CHUNK;
}

__global__ void k_leaf_chunk_count(const int32_t *__restrict__ count, const int32_t *__restrict__ nchild, int32_t nn,
                                   int32_t *__restrict__ out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nn) out[i] = nchild[i] == 0 ? (count[i] + CHUNK - 1) / CHUNK : 0;
}

__device__ inline int32_t node_of_chunk(const int32_t *__restrict__ off, int32_t nn, int32_t ch) {
    int32_t lo = 0, hi = nn;  // last node with off[node] <= ch
    while (hi - lo > 1) {
        const int32_t m = (lo + hi) >> 1;
        if (off[m] <= ch)
            lo = m;
        else
            hi = m;
    }
    return lo;
}

__global__ __launch_bounds__(BT) void k_radius(const double *__restrict__ pos, const int32_t *__restrict__ start,
                                               const int32_t *__restrict__ count, const int32_t *__restrict__ coff,
                                               int32_t nn, const double *__restrict__ center,
                                               double *__restrict__ r2max) {
#pragma clang fp contract(off)
    const int32_t ch = blockIdx.x;
    const int32_t node = node_of_chunk(coff, nn, ch);
    const int32_t first = start[node] + (ch - coff[node]) * CHUNK;
    const int32_t last = min(start[node] + count[node], first + CHUNK);
    const double cx = center[3 * node], cy = center[3 * node + 1], cz = center[3 * node + 2];
    double m = 0.0;
    for (int32_t i = first + threadIdx.x; i < last; i += BT) {
        const double dx = pos[3 * int64_t(i)] - cx;
        const double dy = pos[3 * int64_t(i) + 1] - cy;
        const double dz = pos[3 * int64_t(i) + 2] - cz;
        const double r2 = dx * dx + dy * dy + dz * dz;
        m = fmax(m, r2);
    }
    __shared__ double red[BT];
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_nonneg(&r2max[node], red[0]);
}

// radii from the largest squared distances, the far field's power-of-two scale, and each
// node's traversal record
__global__ void k_radius_final(int32_t nn, double *__restrict__ r, double *__restrict__ rho,
                               const double *__restrict__ center, const int32_t *__restrict__ nchild,
                               const int32_t *__restrict__ child0, const int32_t *__restrict__ count,
                               TravNode *__restrict__ trav) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const double v = sqrt(r[i]);
    r[i] = v;
    rho[i] = rho_of(v);
    TravNode t;
    for (int a = 0; a < 3; ++a) t.c[a] = center[3 * i + a];
    t.r = v;
    t.nchild = nchild[i];
    t.child0 = child0[i];
    t.count = count[i];
    for (int a = 0; a < 5; ++a) t.pad[a] = 0;
    trav[i] = t;
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// grow a node array, keeping its first `keep` bytes
void grow_keep(DBuf &b, size_t keep, size_t want, hipStream_t s) {
    if (want <= b.bytes) return;
    void *np = nullptr;
    STK_HIP(hipMalloc(&np, want));
    if (keep) STK_HIP(hipMemcpyAsync(np, b.p, keep, hipMemcpyDeviceToDevice, s));
    STK_HIP(hipStreamSynchronize(s));
    b.release();
    b.p = np;
    b.bytes = want;
}

}  // namespace

void build_tree(Tree &t, const double *src, int64_t n, int32_t n0, hipStream_t s) {
    t.n = n;
    t.n0 = n0;
    t.have_moments = false;
    prof_mark(-1, s);

    // root cube
    const int nbb = int(std::min<int64_t>(1024, (n + BT - 1) / BT));
    double *part = reserve<double>(t.s_tmp, size_t(nbb) * 6 + 6);
    hipLaunchKernelGGL(k_bounds, dim3(nbb), dim3(BT), 0, s, src, n, part);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(BT), 0, s, part, nbb, part + size_t(nbb) * 6);
    STK_CHECK_LAUNCH();
    double b6[6];
    {
        PeekSrc src[6];
        int64_t raw[6];
        for (int a = 0; a < 6; ++a) src[a] = {part + size_t(nbb) * 6 + a, 8};
        peek(t.peek, s, 6, src, raw);
        std::memcpy(b6, raw, sizeof(b6));
    }
    double L = 0.0;
    for (int a = 0; a < 3; ++a) {
        t.lo[a] = b6[a];
        if (b6[3 + a] - b6[a] > L) L = b6[3 + a] - b6[a];
    }
    t.L = L;
    t.degenerate = !(L > 0.0);
    t.scale = t.degenerate ? 0.0 : 2097152.0 / L;

    // keys, sort, sorted positions
    uint64_t *keys = reserve<uint64_t>(t.keys, size_t(n));
    int32_t *perm = reserve<int32_t>(t.perm, size_t(n));
    hipLaunchKernelGGL(k_keys, dim3(nblk(n, BT)), dim3(BT), 0, s, src, n, t.lo[0], t.lo[1], t.lo[2], t.scale,
                       int(t.degenerate), keys, perm);
    STK_CHECK_LAUNCH();
    radix_sort_pairs(t, keys, perm, n, 63, s);
    double *pos = reserve<double>(t.pos, size_t(n) * 3);
    hipLaunchKernelGGL(k_gather3, dim3(nblk(n, BT)), dim3(BT), 0, s, src, perm, n, pos);
    STK_CHECK_LAUNCH();

    // subdivision, one level per step
    size_t cap = std::max<size_t>(1024, t.nlevel.bytes / sizeof(int32_t));
    for (DBuf *b : {&t.nlevel, &t.nparent, &t.nchild0, &t.nnchild, &t.nstart, &t.ncount}) {
        if (b->bytes < cap * sizeof(int32_t)) {
            b->release();
            b->reserve(cap * sizeof(int32_t));
        }
    }
    // room for every node the top-levels kernel can make
    const size_t top_max = 1 + size_t(STK_MAX_LEVEL) * 8 * TOP_NODES;
    if (!t.degenerate && top_max > cap) {
        size_t ncap = cap;
        while (ncap < top_max) ncap *= 2;
        for (DBuf *b : {&t.nlevel, &t.nparent, &t.nchild0, &t.nnchild, &t.nstart, &t.ncount})
            grow_keep(*b, 0, ncap * sizeof(int32_t), s);
        cap = ncap;
    }
    hipLaunchKernelGGL(k_root, dim3(1), dim3(64), 0, s, int32_t(n), t.nlevel.as<int32_t>(), t.nparent.as<int32_t>(),
                       t.nchild0.as<int32_t>(), t.nnchild.as<int32_t>(), t.nstart.as<int32_t>(),
                       t.ncount.as<int32_t>());
    STK_CHECK_LAUNCH();
    int32_t nnodes = 1, lb = 0, le = 1, lev = 0;
    t.level_begin.assign(1, 0);
    bool complete = t.degenerate;
    if (!t.degenerate) {
        // the sparse top levels in one block, then the host walks the rest level by level
        static_assert(5 + STK_MAX_LEVEL <= PEEK_MAX, "the top kernel's results fit the host slots");
        int64_t *slots = peek_slots(t.peek);
        hipLaunchKernelGGL(k_split_top, dim3(1), dim3(TOP_T), 0, s, keys, int32_t(n), n0, t.nlevel.as<int32_t>(),
                           t.nparent.as<int32_t>(), t.nchild0.as<int32_t>(), t.nnchild.as<int32_t>(),
                           t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), slots);
        STK_CHECK_LAUNCH();
        int64_t r[5 + STK_MAX_LEVEL];
        peek_wait(t.peek, s, 5 + STK_MAX_LEVEL, r);
        for (int64_t j = 0; j < r[0]; ++j) t.level_begin.push_back(int32_t(r[5 + j]));
        lev = int32_t(r[1]);
        lb = int32_t(r[2]);
        le = int32_t(r[3]);
        nnodes = le;
        complete = r[4] != 0;
    }
    while (!complete && lev < STK_MAX_LEVEL) {
        const int32_t nlev = le - lb;
        // room for every child the level can make (at most eight per node), so the
        // children are written before the host reads how many there are
        if (size_t(nnodes) + 8 * size_t(nlev) > cap) {
            size_t ncap = cap;
            while (ncap < size_t(nnodes) + 8 * size_t(nlev)) ncap *= 2;
            for (DBuf *b : {&t.nlevel, &t.nparent, &t.nchild0, &t.nnchild, &t.nstart, &t.ncount})
                grow_keep(*b, size_t(nnodes) * sizeof(int32_t), ncap * sizeof(int32_t), s);
            cap = ncap;
        }
        int32_t *nch = reserve<int32_t>(t.s_vals, size_t(nlev) * 11 + 2);
        int32_t *choff = nch + nlev;
        int32_t *bnd = reserve<int32_t>(t.s_vals2, size_t(nlev) * 9);
        hipLaunchKernelGGL(k_split_count, dim3(nblk(int64_t(nlev) * 64, BT)), dim3(BT), 0, s, keys,
                           t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), lb, nlev, 3 * (STK_MAX_LEVEL - 1 - lev),
                           n0, nch, bnd);
        STK_CHECK_LAUNCH();
        scan_exclusive_i32(nch, choff, nlev, t.s_scan, s);
        hipLaunchKernelGGL(k_split_emit, dim3(nblk(nlev, BT)), dim3(BT), 0, s, lb, nlev, le, lev, nch, choff, bnd,
                           t.nlevel.as<int32_t>(), t.nparent.as<int32_t>(), t.nchild0.as<int32_t>(),
                           t.nnchild.as<int32_t>(), t.nstart.as<int32_t>(), t.ncount.as<int32_t>());
        STK_CHECK_LAUNCH();
        int32_t total = 0;
        {
            const PeekSrc src{choff + nlev, 4};
            int64_t v = 0;
            peek(t.peek, s, 1, &src, &v);
            total = int32_t(v);
        }
        t.level_begin.push_back(le);
        if (total == 0) break;
        nnodes += total;
        lb = le;
        le = nnodes;
        ++lev;
    }
    if (t.level_begin.back() != nnodes) t.level_begin.push_back(nnodes);
    t.nnodes = nnodes;
    t.nlevels = int32_t(t.level_begin.size()) - 1;

    // boxes and centres: leaves from their points, inner nodes from their children
    double *bmin = reserve<double>(t.nbmin, size_t(nnodes) * 3);
    double *bmax = reserve<double>(t.nbmax, size_t(nnodes) * 3);
    double *cen = reserve<double>(t.ncenter, size_t(nnodes) * 3);
    hipLaunchKernelGGL(k_leaf_box, dim3(nnodes), dim3(BT), 0, s, pos, t.nstart.as<int32_t>(),
                       t.ncount.as<int32_t>(), t.nnchild.as<int32_t>(), bmin, bmax, cen);
    STK_CHECK_LAUNCH();
    {
        // levels above `top` are all small: one block takes them, the others a launch each
        int top = t.nlevels - 2;
        int small = -1;  // the deepest level from which every level up to the root is small
        for (int l = 0; l <= top && t.level_begin[l + 1] - t.level_begin[l] <= TOP_BOX_NODES; ++l) small = l;
        for (int l = top; l > small; --l) {
            const int32_t b = t.level_begin[l], e = t.level_begin[l + 1];
            hipLaunchKernelGGL(k_inner_box, dim3(nblk(e - b, BT)), dim3(BT), 0, s, b, e - b,
                               t.nchild0.as<int32_t>(), t.nnchild.as<int32_t>(), bmin, bmax, cen);
            STK_CHECK_LAUNCH();
        }
        if (small >= 0) {
            LevelBegins lv{};
            for (int l = 0; l <= small + 1; ++l) lv.b[l] = t.level_begin[l];
            hipLaunchKernelGGL(k_inner_box_top, dim3(1), dim3(1024), 0, s, small, lv, t.nchild0.as<int32_t>(),
                               t.nnchild.as<int32_t>(), bmin, bmax, cen);
            STK_CHECK_LAUNCH();
        }
    }

    // work chunks and radii
    int32_t *cnt = reserve<int32_t>(t.s_vals, size_t(nnodes));
    int32_t *coff = reserve<int32_t>(t.chunk_off, size_t(nnodes) + 1);
    hipLaunchKernelGGL(k_chunk_count, dim3(nblk(nnodes, BT)), dim3(BT), 0, s, t.ncount.as<int32_t>(), nnodes, cnt);
    STK_CHECK_LAUNCH();
    scan_exclusive_i32(cnt, coff, nnodes, t.s_scan, s);
    int32_t *lcnt = reserve<int32_t>(t.s_vals2, size_t(nnodes));
    int32_t *lcoff = reserve<int32_t>(t.leaf_coff, size_t(nnodes) + 1);
    hipLaunchKernelGGL(k_leaf_chunk_count, dim3(nblk(nnodes, BT)), dim3(BT), 0, s, t.ncount.as<int32_t>(),
                       t.nnchild.as<int32_t>(), nnodes, lcnt);
    STK_CHECK_LAUNCH();
    scan_exclusive_i32(lcnt, lcoff, nnodes, t.s_scan, s);
    double *rad = reserve<double>(t.nradius, size_t(nnodes));
    double *rho = reserve<double>(t.nrho, size_t(nnodes));
    STK_HIP(hipMemsetAsync(rad, 0, sizeof(double) * nnodes, s));
    {
        const PeekSrc src[2] = {{coff + nnodes, 4}, {lcoff + nnodes, 4}};
        int64_t v[2];
        peek(t.peek, s, 2, src, v);
        t.nchunks = int32_t(v[0]);
        t.nleafchunks = int32_t(v[1]);
    }
    hipLaunchKernelGGL(k_radius, dim3(t.nchunks), dim3(BT), 0, s, pos, t.nstart.as<int32_t>(),
                       t.ncount.as<int32_t>(), coff, nnodes, cen, rad);
    STK_CHECK_LAUNCH();
    TravNode *trav = reserve<TravNode>(t.trav, size_t(nnodes));
    hipLaunchKernelGGL(k_radius_final, dim3(nblk(nnodes, BT)), dim3(BT), 0, s, nnodes, rad, rho, cen,
                       t.nnchild.as<int32_t>(), t.nchild0.as<int32_t>(), t.ncount.as<int32_t>(), trav);
    STK_CHECK_LAUNCH();
    prof_mark(STK_PHASE_TREE, s);
}

}  // namespace stk
