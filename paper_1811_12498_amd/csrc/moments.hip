// Cluster moments (Sec. 2) and the per-cluster channel blocks read by the far field.
//
//   M_j^k(C) = sum_{y in C} (y - y_c)^k f_j,   Mt_jl^k(C) = sum_{y in C} (y - y_c)^k h_j nu_l
//
// in FP64.  A leaf's moments are summed directly from its points: work items are (leaf,
// chunk of <= CHUNK points), each writes a partial sum, and the leaf's block in the
// level-by-level pass adds them in chunk order.  An inner node's moments are its children's, moved to its
// centre by the binomial expansion
//   (y - c)^k = sum_{j <= k} C(k, j) (c' - c)^(k - j) (y - c')^j    (c' a child's centre),
// exact in exact arithmetic, level by level from the leaves up; children and terms are
// added in a fixed order, so the result does not depend on scheduling.
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {
namespace {

constexpr int MT = 256;    // threads per block (reduction and block kernels)
constexpr int STAGE = 21;  // points whose powers are tabulated in LDS per round (3 STAGE <= 64 lanes)
constexpr int AMAX = 5;    // multi-indices per lane: 64 * AMAX >= nidx(STK_P_MAX)

__device__ inline int32_t node_of_chunk(const int32_t *__restrict__ off, int32_t nn, int32_t ch) {
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

// One wavefront per (node, chunk of <= CHUNK points) and right-hand side r (grid
// (nchunks, K)).  Lane L owns the multi-indices a = L + 64 j.  The points are taken
// STAGE at a time: the wave stages their powers (y - y_c)_axis^e and their 12 weights
// (f_j, h_j nu_l) in LDS, then for each point each lane adds (y - y_c)^k * weight to its
// 12 accumulators per multi-index.  Powers and the monomial
// are formed by repeated multiplication in the same order as the oracle.
// part[((chunk * K + r) * nm + a) * 12 + c]
template <int A>
__global__ __launch_bounds__(64) void k_moments(const double *__restrict__ pos, const int32_t *__restrict__ start,
                                                const int32_t *__restrict__ count, const int32_t *__restrict__ coff,
                                                int32_t nn, const double *__restrict__ center,
                                                const double *__restrict__ w12, int p, int nm,
                                                double *__restrict__ part) {
    __shared__ double pw[STAGE][3][STK_P_MAX + 1];
    __shared__ double wl[STAGE][12];
    const int32_t ch = blockIdx.x;
    const int r = blockIdx.y;
    const int K = gridDim.y;
    const int lane = threadIdx.x;
    const int32_t node = node_of_chunk(coff, nn, ch);
    const int32_t first = start[node] + (ch - coff[node]) * CHUNK;
    const int32_t last = min(start[node] + count[node], first + CHUNK);
    const double c3[3] = {center[3 * node], center[3 * node + 1], center[3 * node + 2]};
    const int P1 = p + 1;

    int e1[A], e2[A], e3[A];
    double acc[A][12];
#pragma unroll
    for (int j = 0; j < A; ++j) {
        int k[3] = {0, 0, 0};
        if (lane + 64 * j < nm) kof(lane + 64 * j, k);
        e1[j] = k[0];
        e2[j] = k[1];
        e3[j] = k[2];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[j][c] = 0.0;
    }
    for (int32_t b = first; b < last; b += STAGE) {
        const int cnt = min(STAGE, last - b);
        __syncthreads();
        if (lane < 3 * cnt) {  // one lane per (point, axis): d^0 .. d^p by repeated multiplication
            const int pt = lane / 3, ax = lane - 3 * pt;
            const double d = pos[3 * int64_t(b + pt) + ax] - c3[ax];
            double v = 1.0;
            for (int e = 0; e < P1; ++e) {
                pw[pt][ax][e] = v;
                v *= d;
            }
        }
        for (int q = lane; q < 12 * cnt; q += 64) {
            const int pt = q / 12, c = q - 12 * pt;
            wl[pt][c] = w12[(size_t(b + pt) * K + r) * 12 + c];
        }
        __syncthreads();
        for (int pt = 0; pt < cnt; ++pt) {
            double wv[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) wv[c] = wl[pt][c];
#pragma unroll
            for (int j = 0; j < A; ++j) {
                const double mono = pw[pt][0][e1[j]] * pw[pt][1][e2[j]] * pw[pt][2][e3[j]];
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[j][c] += mono * wv[c];
            }
        }
    }
    double *out = part + (size_t(ch) * K + r) * nm * 12;
#pragma unroll
    for (int j = 0; j < A; ++j) {
        const int a = lane + 64 * j;
        if (a < nm)
#pragma unroll
            for (int c = 0; c < 12; ++c) out[a * 12 + c] = acc[j][c];
    }
}

// grid (nodes of one level, K), MT threads, 2 nm * 12 doubles of dynamic LDS; one launch
// per level from the deepest up.  A block first completes its node's moments (an inner
// node: the sum of its children's moments moved to its centre, children in order; a leaf:
// the sum of its chunks' partial moments, in chunk order), then moves them to its parent's
// centre for the level above, one axis at a time,
//   M'(k) = sum_{j <= k_i} C(k_i, j) d_i^(k_i - j) M(k with k_i -> j)   (i = x, y, z),
// which composes to the binomial expansion and keeps every index within ||k|| <= p.  A
// thread takes whole lines along the axis (the other two components and the channel
// fixed): at most p + 1 values in registers and a triangular update.
__device__ inline int m2m_index(int ax, int kl, int u, int v) {
    // multi-index with component ax = kl and the other two (in axis order) = u, v
    return ax == 0 ? gidx(kl, u, v) : (ax == 1 ? gidx(u, kl, v) : gidx(u, v, kl));
}

__global__ __launch_bounds__(MT) void k_m2m(const double *__restrict__ center, const int32_t *__restrict__ child0,
                                            const int32_t *__restrict__ nchild, const int32_t *__restrict__ parent,
                                            const double *__restrict__ part, const int32_t *__restrict__ leaf_coff,
                                            int32_t lev_begin, int p, int nm, double *__restrict__ mom,
                                            double *__restrict__ up) {
    extern __shared__ double m2m_lds[];
    __shared__ double fac[3][STK_P_MAX + 1][STK_P_MAX + 1];  // C(k, j) d^(k - j) per axis
    const int32_t node = lev_begin + blockIdx.x;
    const int r = blockIdx.y, K = gridDim.y;
    const int tid = threadIdx.x;
    const int nq = nm * 12;
    double *buf0 = m2m_lds, *buf1 = m2m_lds + nq;
    auto at = [&](int32_t nd, int q) { return (size_t(nd) * nm + q / 12) * 12 * K + 12 * r + q % 12; };
    const int nc = nchild[node];
    if (nc > 0) {
        const int32_t c0 = child0[node];
        for (int q = tid; q < nq; q += MT) {
            double s = 0.0;
            for (int ci = 0; ci < nc; ++ci) s += up[at(c0 + ci, q)];
            mom[at(node, q)] = s;
            buf0[q] = s;
        }
    } else {
        // part[((chunk * K + r) * nm + a) * 12 + c], the leaf's chunks c0 .. c1 - 1
        const int32_t c0 = leaf_coff[node], c1 = leaf_coff[node + 1];
        const size_t stride = size_t(K) * nm * 12;
        for (int q = tid; q < nq; q += MT) {
            const double *src = part + (size_t(c0) * K + r) * nm * 12 + q;
            double v = 0.0;
            for (int32_t ch = c0; ch < c1; ++ch, src += stride) v += *src;
            mom[at(node, q)] = v;
            buf0[q] = v;
        }
    }
    const int32_t par = parent[node];
    if (par < 0) return;  // the root
    if (tid < 3) {
        // row k: C(k, j) d^(k - j), with C(k, j) = C(k - 1, j - 1) + C(k - 1, j)
        const double d = center[3 * node + tid] - center[3 * par + tid];
        double dp[STK_P_MAX + 1];
        dp[0] = 1.0;
        for (int e = 1; e <= p; ++e) dp[e] = dp[e - 1] * d;
        double bin[STK_P_MAX + 1];
        for (int k = 0; k <= p; ++k) {
            bin[k] = 1.0;
            for (int j = k - 1; j > 0; --j) bin[j] += bin[j - 1];
            for (int j = 0; j <= k; ++j) fac[tid][k][j] = bin[j] * dp[k - j];
        }
    }
    const int nline = (p + 1) * (p + 2) / 2 * 12;  // (u, v) with u + v <= p, channel
    for (int ax = 0; ax < 3; ++ax) {
        __syncthreads();
        const double *in = ax == 1 ? buf1 : buf0;
        double *out = ax == 0 ? buf1 : buf0;
        for (int ln = tid; ln < nline; ln += MT) {
            const int c = ln % 12, pr = ln / 12;
            // pair pr -> (u, v): u + v = s, v = pr - s (s + 1) / 2
            int sv = 0;
            while ((sv + 1) * (sv + 2) / 2 <= pr) ++sv;
            const int v = pr - sv * (sv + 1) / 2, u = sv - v;
            const int len = p - sv + 1;  // kl = 0 .. p - u - v
            double x[STK_P_MAX + 1];
#pragma unroll
            for (int kl = 0; kl <= STK_P_MAX; ++kl) x[kl] = kl < len ? in[m2m_index(ax, kl, u, v) * 12 + c] : 0.0;
#pragma unroll
            for (int kl = 0; kl <= STK_P_MAX; ++kl) {
                if (kl < len) {
                    double y = 0.0;
#pragma unroll
                    for (int jj = 0; jj <= kl; ++jj) y += fac[ax][kl][jj] * x[jj];
                    const int o = m2m_index(ax, kl, u, v) * 12 + c;
                    if (ax == 2)
                        up[at(node, o)] = y;
                    else
                        out[o] = y;
                }
            }
        }
    }
}

// grid (nnodes, K): each cluster's far-field stream (stk_math.hpp) in the evaluation
// precision, wblk[(node * K + r) * 6 nG + pos], nG = nidx(p + 1)
// The cluster's 12 nm moments of this right-hand side are staged in LDS first (every
// value is read by many outputs).
template <typename T>
__global__ __launch_bounds__(MT) void k_channels(const double *__restrict__ mom, const double *__restrict__ rho, int p,
                                                 int nm, int ng, T *__restrict__ wblk) {
    extern __shared__ double ms[];  // [nm][12]
    const int32_t node = blockIdx.x;
    const int r = blockIdx.y, K = gridDim.y;
    const double *src = mom + size_t(node) * nm * 12 * K + 12 * r;
    for (int i = threadIdx.x; i < 12 * nm; i += MT) {
        const int a = i / 12;
        ms[i] = src[size_t(a) * 12 * K + (i - 12 * a)];
    }
    __syncthreads();
    const double inv = 1.0 / rho[node];  // a power of two: exact
    T *out = wblk + (size_t(node) * K + r) * 6 * ng;
    for (int a = threadIdx.x; a < ng; a += MT) {
        int q[3];
        kof(a, q);
        double ge[6];
        phi_ge(ms, 12, p, q, ge);
        double s = 1.0;
        for (int e = 0; e < q[0] + q[1] + q[2]; ++e) s *= inv;
        int pg, pe;
        stream_pos(p, q, pg, pe);
        for (int c = 0; c < 3; ++c) {
            out[pg + c] = T(ge[c] * s);
            out[pe + c] = T(ge[3 + c] * s * inv);
        }
    }
}

// per-source records in Morton order: geo = (y, nu) FP64 and wts = (f, h) per RHS in the
// evaluation precision (near field); w12 = (f_j, h_j nu_l) per RHS in FP64 (moments)
template <typename T>
__global__ void k_records(const double *__restrict__ pos, const int32_t *__restrict__ perm, int64_t n, int K,
                          const double *__restrict__ f, const double *__restrict__ h, const double *__restrict__ nu,
                          double *__restrict__ geo, T *__restrict__ wts, double *__restrict__ w12) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    double nv[3];
    for (int a = 0; a < 3; ++a) {
        nv[a] = nu[3 * j + a];
        geo[6 * i + a] = pos[3 * i + a];
        geo[6 * i + 3 + a] = nv[a];
    }
    for (int r = 0; r < K; ++r) {
        double fv[3], hv[3];
        for (int a = 0; a < 3; ++a) {
            fv[a] = f[(size_t(r) * n + j) * 3 + a];
            hv[a] = h[(size_t(r) * n + j) * 3 + a];
            wts[(i * K + r) * 6 + a] = T(fv[a]);
            wts[(i * K + r) * 6 + 3 + a] = T(hv[a]);
        }
        double *w = w12 + (i * K + r) * 12;
        for (int a = 0; a < 3; ++a) w[a] = fv[a];
        for (int jj = 0; jj < 3; ++jj)
            for (int l = 0; l < 3; ++l) w[3 + 3 * jj + l] = hv[jj] * nv[l];
    }
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

// direct moments of the leaves (their chunks only)
template <int A>
static void launch_moments(Tree &t, int K, int p, int nm, const double *w12, double *part, hipStream_t s) {
    if (t.nleafchunks == 0) return;
    hipLaunchKernelGGL(k_moments<A>, dim3(t.nleafchunks, K), dim3(64), 0, s, t.pos.as<double>(),
                       t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), t.leaf_coff.as<int32_t>(), t.nnodes,
                       t.ncenter.as<double>(), w12, p, nm, part);
    STK_CHECK_LAUNCH();
}

void compute_moments(Tree &t, const double *f, const double *h, const double *nu, int32_t K, int32_t p,
                     stk_precision prec, hipStream_t s, hipEvent_t records_done) {
    const int nm = nidx(p), ng = nidx(p + 1);
    const int32_t nn = t.nnodes;
    prof_mark(-1, s);
    const size_t esz = prec == STK_FP64 ? sizeof(double) : sizeof(float);
    t.wblk.reserve(size_t(nn) * ng * 6 * K * esz);
    t.geo.reserve(size_t(t.n) * 6 * sizeof(double));
    t.wts.reserve(size_t(t.n) * K * 6 * esz);
    double *w12 = reserve<double>(t.w12, size_t(t.n) * K * 12);
    if (prec == STK_FP64)
        hipLaunchKernelGGL(k_records<double>, dim3(nblk(t.n, 256)), dim3(256), 0, s, t.pos.as<double>(),
                           t.perm.as<int32_t>(), t.n, K, f, h, nu, t.geo.as<double>(), t.wts.as<double>(), w12);
    else
        hipLaunchKernelGGL(k_records<float>, dim3(nblk(t.n, 256)), dim3(256), 0, s, t.pos.as<double>(),
                           t.perm.as<int32_t>(), t.n, K, f, h, nu, t.geo.as<double>(), t.wts.as<float>(), w12);
    STK_CHECK_LAUNCH();
    if (records_done) STK_HIP(hipEventRecord(records_done, s));

    double *part = reserve<double>(t.mom_part, size_t(t.nleafchunks) * K * nm * 12 + 1);
    const int A = (nm + 63) / 64;
    switch (A) {
        case 1: launch_moments<1>(t, K, p, nm, w12, part, s); break;
        case 2: launch_moments<2>(t, K, p, nm, w12, part, s); break;
        case 3: launch_moments<3>(t, K, p, nm, w12, part, s); break;
        case 4: launch_moments<4>(t, K, p, nm, w12, part, s); break;
        case 5: launch_moments<5>(t, K, p, nm, w12, part, s); break;
        default: throw Error(STK_EINVAL, "p too large for the moment kernel");
    }
    double *mom = reserve<double>(t.mom, size_t(nn) * nm * 12 * K);
    // every level from the deepest up: complete inner nodes from their children, move each
    // node's moments to its parent's centre
    double *up = reserve<double>(t.mom_up, size_t(nn) * nm * 12 * K);
    for (int l = t.nlevels - 1; l >= 0; --l) {
        const int32_t b = t.level_begin[l], e = t.level_begin[l + 1];
        if (e > b) {
            hipLaunchKernelGGL(k_m2m, dim3(e - b, K), dim3(MT), sizeof(double) * 2 * nm * 12, s,
                               t.ncenter.as<double>(), t.nchild0.as<int32_t>(), t.nnchild.as<int32_t>(),
                               t.nparent.as<int32_t>(), part, t.leaf_coff.as<int32_t>(), b, p, nm, mom, up);
            STK_CHECK_LAUNCH();
        }
    }
    if (prec == STK_FP64)
        hipLaunchKernelGGL(k_channels<double>, dim3(nn, K), dim3(MT), sizeof(double) * 12 * nm, s, mom, t.nrho.as<double>(), p, nm, ng,
                           t.wblk.as<double>());
    else
        hipLaunchKernelGGL(k_channels<float>, dim3(nn, K), dim3(MT), sizeof(double) * 12 * nm, s, mom, t.nrho.as<double>(), p, nm, ng,
                           t.wblk.as<float>());
    STK_CHECK_LAUNCH();
    prof_mark(STK_PHASE_MOMENTS, s);
    t.p = p;
    t.k_rhs = K;
    t.prec = prec;
    t.have_moments = true;
}

}  // namespace stk
