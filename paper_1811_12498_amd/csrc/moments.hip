// Cluster moments (Sec. 2) and the per-cluster channel blocks read by the far field.
//
//   M_j^k(C) = sum_{y in C} (y - y_c)^k f_j,   Mt_jl^k(C) = sum_{y in C} (y - y_c)^k h_j nu_l
//
// computed directly from each node's points (every point contributes to each of its
// ancestors), in FP64.  Work items are (node, chunk of <= CHUNK points); each item
// writes a partial sum and a second kernel adds a node's partials in chunk order, so
// the result does not depend on scheduling.
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {
namespace {

constexpr int MT = 256;    // threads per block
constexpr int STAGE = 32;  // points staged in LDS per round

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

// grid (nchunks, K).  part[((chunk * K + r) * nm + a) * 12 + c]
__global__ __launch_bounds__(MT) void k_moments(const double *__restrict__ pos, const int32_t *__restrict__ perm,
                                                const int32_t *__restrict__ start, const int32_t *__restrict__ count,
                                                const int32_t *__restrict__ coff, int32_t nn,
                                                const double *__restrict__ center, const double *__restrict__ f,
                                                const double *__restrict__ h, const double *__restrict__ nu, int64_t n,
                                                int p, int nm, double *__restrict__ part) {
    extern __shared__ double sm[];
    const int P1 = p + 1;
    double *pw = sm;                      // [STAGE][3][P1] powers of y - y_c
    double *wt = sm + STAGE * 3 * P1;     // [STAGE][12] f_j and h_j nu_l
    const int32_t ch = blockIdx.x;
    const int r = blockIdx.y;
    const int K = gridDim.y;
    const int32_t node = node_of_chunk(coff, nn, ch);
    const int32_t first = start[node] + (ch - coff[node]) * CHUNK;
    const int32_t last = min(start[node] + count[node], first + CHUNK);
    const double cx = center[3 * node], cy = center[3 * node + 1], cz = center[3 * node + 2];

    // each thread owns up to two multi-indices
    int ka[2][3];
    const int a0 = threadIdx.x, a1 = threadIdx.x + MT;
    if (a0 < nm) kof(a0, ka[0]);
    if (a1 < nm) kof(a1, ka[1]);
    double acc[2][12];
    for (int u = 0; u < 2; ++u)
        for (int c = 0; c < 12; ++c) acc[u][c] = 0.0;

    const double *fr = f + size_t(r) * n * 3;
    const double *hr = h + size_t(r) * n * 3;
    for (int32_t b = first; b < last; b += STAGE) {
        const int cnt = min(STAGE, last - b);
        __syncthreads();
        for (int q = threadIdx.x; q < cnt * 3; q += MT) {
            const int j = q / 3, ax = q % 3;
            const double c = ax == 0 ? cx : (ax == 1 ? cy : cz);
            const double d = pos[3 * int64_t(b + j) + ax] - c;
            double *row = pw + (j * 3 + ax) * P1;
            double v = 1.0;
            row[0] = 1.0;
            for (int e = 1; e <= p; ++e) {
                v *= d;
                row[e] = v;
            }
        }
        for (int q = threadIdx.x; q < cnt * 12; q += MT) {
            const int j = q / 12, c = q % 12;
            const int64_t src = perm[b + j];
            double w;
            if (c < 3)
                w = fr[3 * src + c];
            else
                w = hr[3 * src + (c - 3) / 3] * nu[3 * src + (c - 3) % 3];
            wt[j * 12 + c] = w;
        }
        __syncthreads();
        for (int u = 0; u < 2; ++u) {
            if ((u == 0 ? a0 : a1) >= nm) continue;
            const int k1 = ka[u][0], k2 = ka[u][1], k3 = ka[u][2];
            for (int j = 0; j < cnt; ++j) {
                const double mono = pw[(j * 3) * P1 + k1] * pw[(j * 3 + 1) * P1 + k2] * pw[(j * 3 + 2) * P1 + k3];
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[u][c] += mono * wt[j * 12 + c];
            }
        }
    }
    double *out = part + (size_t(ch) * K + r) * nm * 12;
    for (int u = 0; u < 2; ++u) {
        const int a = u == 0 ? a0 : a1;
        if (a >= nm) continue;
        for (int c = 0; c < 12; ++c) out[a * 12 + c] = acc[u][c];
    }
}

// grid (nnodes, K): mom[(node * nm + a) * 12K + 12 r + c] = sum over the node's chunks
__global__ __launch_bounds__(MT) void k_moments_reduce(const double *__restrict__ part, const int32_t *__restrict__ coff,
                                                       int nm, double *__restrict__ mom) {
    const int32_t node = blockIdx.x;
    const int r = blockIdx.y, K = gridDim.y;
    const int32_t c0 = coff[node], c1 = coff[node + 1];
    for (int q = threadIdx.x; q < nm * 12; q += MT) {
        double s = 0.0;
        for (int32_t ch = c0; ch < c1; ++ch) s += part[(size_t(ch) * K + r) * nm * 12 + q];
        const int a = q / 12, c = q % 12;
        mom[(size_t(node) * nm + a) * 12 * K + 12 * r + c] = s;
    }
}

// grid (nnodes, K): far-field blocks for ||a|| <= p + 1 in the evaluation precision,
// wblk[(node * K + r) * 6 nG + 3a + i] = G_i^a / rho^||a||  and
// wblk[(node * K + r) * 6 nG + 3 nG + 3a + l] = E_l^a / rho^(||a||+1)
template <typename T>
__global__ __launch_bounds__(MT) void k_channels(const double *__restrict__ mom, const double *__restrict__ rho, int p,
                                                 int nm, int ng, T *__restrict__ wblk) {
    const int32_t node = blockIdx.x;
    const int r = blockIdx.y, K = gridDim.y;
    const double inv = 1.0 / rho[node];  // a power of two: exact
    T *out = wblk + (size_t(node) * K + r) * 6 * ng;
    for (int a = threadIdx.x; a < ng; a += MT) {
        int q[3];
        kof(a, q);
        double ge[6];
        phi_ge(mom + size_t(node) * nm * 12 * K + 12 * r, 12 * K, p, q, ge);
        double s = 1.0;
        for (int e = 0; e < q[0] + q[1] + q[2]; ++e) s *= inv;
        for (int c = 0; c < 3; ++c) {
            out[3 * a + c] = T(ge[c] * s);
            out[3 * ng + 3 * a + c] = T(ge[3 + c] * s * inv);
        }
    }
}

// near-field source records in Morton order: geo = (y, nu) FP64; wts = (f, h) per RHS
template <typename T>
__global__ void k_records(const double *__restrict__ pos, const int32_t *__restrict__ perm, int64_t n, int K,
                          const double *__restrict__ f, const double *__restrict__ h, const double *__restrict__ nu,
                          double *__restrict__ geo, T *__restrict__ wts) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    for (int a = 0; a < 3; ++a) {
        geo[6 * i + a] = pos[3 * i + a];
        geo[6 * i + 3 + a] = nu[3 * j + a];
    }
    for (int r = 0; r < K; ++r)
        for (int a = 0; a < 3; ++a) {
            wts[(i * K + r) * 6 + a] = T(f[(size_t(r) * n + j) * 3 + a]);
            wts[(i * K + r) * 6 + 3 + a] = T(h[(size_t(r) * n + j) * 3 + a]);
        }
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

void compute_moments(Tree &t, const double *f, const double *h, const double *nu, int32_t K, int32_t p,
                     stk_precision prec, hipStream_t s) {
    const int nm = nidx(p), ng = nidx(p + 1);
    const int32_t nn = t.nnodes;
    prof_mark(-1, s);
    double *part = reserve<double>(t.s_tmp, size_t(t.nchunks) * K * nm * 12);
    const size_t shm = sizeof(double) * STAGE * (3 * (p + 1) + 12);
    hipLaunchKernelGGL(k_moments, dim3(t.nchunks, K), dim3(MT), shm, s, t.pos.as<double>(), t.perm.as<int32_t>(),
                       t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), t.chunk_off.as<int32_t>(), nn,
                       t.ncenter.as<double>(), f, h, nu, t.n, p, nm, part);
    STK_CHECK_LAUNCH();
    double *mom = reserve<double>(t.mom, size_t(nn) * nm * 12 * K);
    hipLaunchKernelGGL(k_moments_reduce, dim3(nn, K), dim3(MT), 0, s, part, t.chunk_off.as<int32_t>(), nm, mom);
    STK_CHECK_LAUNCH();
    const size_t esz = prec == STK_FP64 ? sizeof(double) : sizeof(float);
    t.wblk.reserve(size_t(nn) * ng * 6 * K * esz);
    t.geo.reserve(size_t(t.n) * 6 * sizeof(double));
    t.wts.reserve(size_t(t.n) * K * 6 * esz);
    if (prec == STK_FP64) {
        hipLaunchKernelGGL(k_channels<double>, dim3(nn, K), dim3(MT), 0, s, mom, t.nrho.as<double>(), p, nm, ng,
                           t.wblk.as<double>());
        STK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_records<double>, dim3(nblk(t.n, 256)), dim3(256), 0, s, t.pos.as<double>(),
                           t.perm.as<int32_t>(), t.n, K, f, h, nu, t.geo.as<double>(), t.wts.as<double>());
    } else {
        hipLaunchKernelGGL(k_channels<float>, dim3(nn, K), dim3(MT), 0, s, mom, t.nrho.as<double>(), p, nm, ng,
                           t.wblk.as<float>());
        STK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_records<float>, dim3(nblk(t.n, 256)), dim3(256), 0, s, t.pos.as<double>(),
                           t.perm.as<int32_t>(), t.n, K, f, h, nu, t.geo.as<double>(), t.wts.as<float>());
    }
    STK_CHECK_LAUNCH();
    prof_mark(STK_PHASE_MOMENTS, s);
    t.p = p;
    t.k_rhs = K;
    t.prec = prec;
    t.have_moments = true;
}

}  // namespace stk
