// Adjoint of the frozen-plan treecode operator: gradients of L = sum_m w^m . u^m with
// respect to f, h, source positions and target positions, with the interaction lists,
// cluster membership, centres, radii and scales of the forward evaluation held fixed.
//
//   near field   target side: d/dx of every near pair (analytic derivative of the
//                contracted pair of Sec. 4.1); source side: the same pairs gathered per
//                source through leaf-major (transposed) near lists.
//   far field    target side: k_far_tgrad (adjoint_far.hpp); source side: per-cluster
//                stream adjoints Lambda_C (k_far_lambda) -> moment adjoints through the
//                transpose of the moment-to-stream map -> per source
//                  dL/df_j  = sum_C sum_k (y - y_c)^k dL/dM_j^k(C)
//                  dL/dh_j  = sum_C sum_k (y - y_c)^k sum_l nu_l dL/dMt_jl^k(C)
//                  dL/dy_s  = sum_C sum_k k_s (y - y_c)^{k - e_s} [f . dL/dM^k + (h nu) : dL/dMt^k]
//                (each source in one node per level: per-level partial sums, then a
//                fixed-order total).
#include <map>
#include <mutex>

#include "adjoint_far.hpp"
#include "lists.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {


namespace {

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// incidences per cluster-adjoint work item (16 passes of 64 lanes): the item's LDS
// accumulator is added to the cluster's stream adjoint once, with atomics, at its end
constexpr int32_t LAMBDA_RUN = 16 * 64;

// ---- near-field adjoint ------------------------------------------------------------------
// dL/dx of one pair (w.u, u the contracted pair of Sec. 4.1) in FP64
__device__ inline void pgrad_f64(const double d[3], const double f[3], const double h[3], const double nu[3],
                                 const double w[3], double gx[3]) {
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double ri = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double r2i = ri * ri, r3i = ri * r2i, r5i = r3i * r2i;
    const double df = d[0] * f[0] + d[1] * f[1] + d[2] * f[2];
    const double dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
    const double dn = d[0] * nu[0] + d[1] * nu[1] + d[2] * nu[2];
    const double wd = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
    const double wf = w[0] * f[0] + w[1] * f[1] + w[2] * f[2];
    const double s = df * r3i, tt = dh * dn * r5i;
    // gx = -wf d r3i + w (s + tt) + wd (f r3i - 3 s d r2i + (h dn + dh nu) r5i - 5 tt d r2i),
    // gathered per vector: five pair scalars, then five multiply-adds per component
    const double A = -(wf * r3i + (wd * r2i) * (3.0 * s + 5.0 * tt)), B = s + tt, C = wd * r3i;
    const double W5 = wd * r5i, D = W5 * dn, E = W5 * dh;
    for (int q = 0; q < 3; ++q) gx[q] = d[q] * A + w[q] * B + f[q] * C + h[q] * D + nu[q] * E;
}

// mixed precision: d and d.nu arrive in FP64, the rest in FP32
__device__ inline void pgrad_mixed(const double dd[3], double dnd, const float f[3], const float h[3],
                                   const double nu64[3], const float w[3], float gx[3]) {
    const float d[3] = {float(dd[0]), float(dd[1]), float(dd[2])};
    const float nu[3] = {float(nu64[0]), float(nu64[1]), float(nu64[2])};
    const float r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float ri = r2 > 0.0f ? __frsqrt_rn(r2) : 0.0f;
    const float r2i = ri * ri, r3i = ri * r2i, r5i = r3i * r2i;
    const float df = d[0] * f[0] + d[1] * f[1] + d[2] * f[2];
    const float dh = d[0] * h[0] + d[1] * h[1] + d[2] * h[2];
    const float dn = float(dnd);
    const float wd = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
    const float wf = w[0] * f[0] + w[1] * f[1] + w[2] * f[2];
    const float s = df * r3i, tt = dh * dn * r5i;
    // the expression of pgrad_f64, gathered the same way
    const float A = -(wf * r3i + (wd * r2i) * (3.0f * s + 5.0f * tt)), B = s + tt, C = wd * r3i;
    const float W5 = wd * r5i, D = W5 * dn, E = W5 * dh;
    for (int q = 0; q < 3; ++q) gx[q] = d[q] * A + w[q] * B + f[q] * C + h[q] * D + nu[q] * E;
}

struct NearAdjArgs {
    const double *tpos, *ws;
    int64_t m;
    const int32_t *off, *node;   // group-major near lists
    const uint64_t *mask;
    const int32_t *start, *count;
    const double *geo;           // (n,6) y, nu
    const void *wts;             // (n,6) f, h in T
    double *gt;                  // (m,3) sorted: near part of dL/dx
    // source side
    const int32_t *item_node, *item_j0;  // work item -> leaf, first source
    const int32_t *ent, *ent_off;        // leaf-sorted near entries; per-leaf offsets
    const int32_t *ent_group;
    double *gs;                  // (n, 9) sorted: near part of dL/df, dL/dh, dL/dy
    int32_t nitems;
};

// target side, leaf major (the forward plan's near work items): one wave per item, a
// leaf against up to 64 of its targets; each incidence's partial gradient goes to its
// slot in the target's near list, and k_slot_reduce adds the slots in list order (the
// same sums, in the same order, as a walk of each target's own list)
struct NearTgradArgs {
    const double *tpos, *ws;
    const int32_t *item_leaf, *item_i0, *item_i1;
    const int32_t *inc_tgt, *inc_slot;
    const int32_t *start, *count;
    const double *geo;           // (n,6) y, nu
    const void *wts;             // (n,6) f, h in T
    void *part;                  // (incidences, 3) T
    int32_t nitems;
};

template <typename T> __global__ __launch_bounds__(64) void k_near_tgrad(NearTgradArgs a) {
    const int32_t it = xcd_item<XCD_CHUNK_NEAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    const int32_t c = a.item_leaf[it];
    const int32_t i0 = a.item_i0[it];
    const bool on = lane < a.item_i1[it] - i0;
    int32_t slot = 0;
    double x[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    if (on) {
        const int64_t t = a.inc_tgt[i0 + lane];
        slot = a.inc_slot[i0 + lane];
        for (int q = 0; q < 3; ++q) {
            x[q] = a.tpos[3 * t + q];
            w[q] = a.ws[3 * t + q];
        }
    }
    // read-only source records through the constant address space (scalar loads)
    const STK_CONST_AS double *geo = (const STK_CONST_AS double *)(a.geo);
    const STK_CONST_AS T *wts = (const STK_CONST_AS T *)(a.wts);
    const float wf[3] = {float(w[0]), float(w[1]), float(w[2])};
    T s0 = T(0), s1 = T(0), s2 = T(0);
    const int32_t j0 = a.start[c], j1 = j0 + a.count[c];
    for (int32_t j = j0; j < j1; ++j) {
        double gj[6];
        T wj[6];
        for (int q = 0; q < 6; ++q) {
            gj[q] = geo[6 * int64_t(j) + q];
            wj[q] = wts[6 * int64_t(j) + q];
        }
        const double d[3] = {x[0] - gj[0], x[1] - gj[1], x[2] - gj[2]};
        if constexpr (sizeof(T) == 8) {
            double gx[3];
            pgrad_f64(d, reinterpret_cast<const double *>(wj), reinterpret_cast<const double *>(wj) + 3, gj + 3, w, gx);
            s0 += gx[0];
            s1 += gx[1];
            s2 += gx[2];
        } else {
            const double dn = d[0] * gj[3] + d[1] * gj[4] + d[2] * gj[5];
            float gx[3];
            pgrad_mixed(d, dn, reinterpret_cast<const float *>(wj), reinterpret_cast<const float *>(wj) + 3, gj + 3,
                        wf, gx);
            s0 += gx[0];
            s1 += gx[1];
            s2 += gx[2];
        }
    }
    if (on) {
        T *o = static_cast<T *>(a.part) + 3 * int64_t(slot);
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

// per target: its slots in near-list order, compensated, to FP64 (m,3)
template <typename T>
__global__ void k_slot_reduce(const T *__restrict__ part, const int32_t *__restrict__ toff, int64_t m,
                              double *__restrict__ out) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= m) return;
    Comp<T> acc[3];
    for (int32_t k = toff[t]; k < toff[t + 1]; ++k)
        for (int q = 0; q < 3; ++q) acc[q].add(part[3 * int64_t(k) + q]);
    for (int q = 0; q < 3; ++q) out[3 * t + q] = acc[q].value();
}

// one source per lane, SG_WAVES waves per block on the same 64 sources: wave w loops over
// the w-th quarter of the leaf's near entries (in order) and the targets of each; the
// waves' partial sums are added in wave order
constexpr int SG_WAVES = 4;
template <typename T> __global__ __launch_bounds__(64 * SG_WAVES) void k_near_sgrad(NearAdjArgs a) {
    __shared__ double red[SG_WAVES - 1][9][64];
    const int32_t it = blockIdx.x;
    if (it >= a.nitems) return;
    // the wave index made visibly wave-uniform: the entry range, masks and target loads of
    // the loop below then stay scalar
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / 64)), lane = threadIdx.x % 64;
    const int32_t c = a.item_node[it];
    const int32_t j = a.item_j0[it] + lane;
    const bool valid = j < a.start[c] + a.count[c];
    const int32_t jj = valid ? j : a.start[c];
    double y[3], nu[3];
    for (int q = 0; q < 3; ++q) {
        y[q] = a.geo[6 * int64_t(jj) + q];
        nu[q] = a.geo[6 * int64_t(jj) + 3 + q];
    }
    const T *wj = static_cast<const T *>(a.wts) + 6 * int64_t(jj);
    const T f[3] = {wj[0], wj[1], wj[2]}, h[3] = {wj[3], wj[4], wj[5]};
    Comp<T> af[3], ah[3], ay[3];
    const int64_t ne = a.ent_off[c + 1] - a.ent_off[c];
    const int32_t eb = a.ent_off[c] + int32_t(ne * wv / SG_WAVES), ee = a.ent_off[c] + int32_t(ne * (wv + 1) / SG_WAVES);
    for (int32_t e = eb; e < ee; ++e) {
        const int32_t ent = a.ent[e];
        const int32_t g = a.ent_group[ent];
        uint64_t mk = a.mask[ent];
        T sf[3] = {T(0), T(0), T(0)}, sh[3] = {T(0), T(0), T(0)}, sy[3] = {T(0), T(0), T(0)};
        while (mk) {
            const int b = __builtin_ctzll(mk);
            mk &= mk - 1;
            const int64_t t = int64_t(g) * 64 + b;
            const double x[3] = {a.tpos[3 * t], a.tpos[3 * t + 1], a.tpos[3 * t + 2]};
            const double wd64[3] = {a.ws[3 * t], a.ws[3 * t + 1], a.ws[3 * t + 2]};
            const double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
            const double dn = d[0] * nu[0] + d[1] * nu[1] + d[2] * nu[2];
            const T dt[3] = {T(d[0]), T(d[1]), T(d[2])};
            const T wv[3] = {T(wd64[0]), T(wd64[1]), T(wd64[2])};
            const T r2 = dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2];
            T ri = T(0);
            if constexpr (sizeof(T) == 8) {
                const double r2d = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                ri = T(r2d > 0.0 ? rsqrt(r2d) : 0.0);
            } else {
                ri = r2 > T(0) ? T(__frsqrt_rn(float(r2))) : T(0);
            }
            const T r3i = ri * ri * ri, r5i = r3i * ri * ri;
            const T wdot = wv[0] * dt[0] + wv[1] * dt[1] + wv[2] * dt[2];
            // dL/df: w ri + (w.d) r3i d; dL/dh: (w.d)(d.nu) r5i d, as multiply-adds per component
            const T a3 = wdot * r3i, a5 = wdot * T(dn) * r5i;
            for (int q = 0; q < 3; ++q) {
                sf[q] += wv[q] * ri + a3 * dt[q];
                sh[q] += a5 * dt[q];
            }
            T gx[3];
            if constexpr (sizeof(T) == 8) {
                double gx64[3];
                pgrad_f64(d, reinterpret_cast<const double *>(f), reinterpret_cast<const double *>(h), nu, wd64, gx64);
                for (int q = 0; q < 3; ++q) gx[q] = T(gx64[q]);
            } else {
                float gx32[3];
                pgrad_mixed(d, dn, reinterpret_cast<const float *>(f), reinterpret_cast<const float *>(h), nu,
                            reinterpret_cast<const float *>(wv), gx32);
                for (int q = 0; q < 3; ++q) gx[q] = T(gx32[q]);
            }
            for (int q = 0; q < 3; ++q) sy[q] -= gx[q];
        }
        for (int q = 0; q < 3; ++q) {
            af[q].add(sf[q]);
            ah[q].add(sh[q]);
            ay[q].add(sy[q]);
        }
    }
    double v[9];
    for (int q = 0; q < 3; ++q) {
        v[q] = af[q].value();
        v[3 + q] = ah[q].value();
        v[6 + q] = ay[q].value();
    }
    if (wv > 0)
        for (int q = 0; q < 9; ++q) red[wv - 1][q][lane] = v[q];
    __syncthreads();
    if (wv == 0 && valid) {
        double *o = a.gs + 9 * int64_t(j);
        for (int q = 0; q < 9; ++q) {
            double s = v[q];
            for (int w = 0; w < SG_WAVES - 1; ++w) s += red[w][q][lane];
            o[q] = s;
        }
    }
}

// ---- moment adjoints: transpose of the moment -> stream map ------------------------------
struct PhiT {
    int p = -1;
    DBuf col_off, rowpos, epow;  // int32
    DBuf coef;                   // double
    DBuf cpos, ckind;            // int32 (columns) for k_far_lambda
};

std::mutex g_phit_mu;
std::map<std::pair<int, int>, PhiT *> g_phit;  // (device, p) -> table; kept for the process

// Sparse matrix S with stream[pos] = sum S[pos, (a, c)] M[a][c] / rho^epow[pos], stored
// by moment column, built once per order from phi_ge applied to unit moments.
PhiT &phit_for(int dev, int p) {
    std::lock_guard<std::mutex> lk(g_phit_mu);
    auto key = std::make_pair(dev, p);
    auto itr = g_phit.find(key);
    if (itr != g_phit.end()) return *itr->second;
    const int nm = nidx(p), ng = nidx(p + 1);
    std::vector<int32_t> col_off(12 * nm + 1, 0), rowpos, epow(6 * ng, 0);
    std::vector<double> coef;
    std::vector<double> mom(size_t(nm) * 12, 0.0);
    for (int b = 0; b < ng; ++b) {
        int q[3], pg, pe;
        kof(b, q);
        stream_pos(p, q, pg, pe);
        const int n = q[0] + q[1] + q[2];
        for (int c = 0; c < 3; ++c) {
            epow[pg + c] = n;
            epow[pe + c] = n + 1;
        }
    }
    for (int a = 0; a < nm; ++a) {
        int ka[3];
        kof(a, ka);
        const int na = ka[0] + ka[1] + ka[2];
        for (int c = 0; c < 12; ++c) {
            mom[size_t(a) * 12 + c] = 1.0;
            // only multi-indices of order na .. na + 2 read moment a
            const int b0 = na > 0 ? nidx(na - 1) : 0, b1 = nidx(std::min(na + 2, p + 1));
            for (int b = b0; b < b1; ++b) {
                int q[3], pg, pe;
                kof(b, q);
                double ge[6];
                phi_ge(mom.data(), 12, p, q, ge);
                stream_pos(p, q, pg, pe);
                for (int k = 0; k < 6; ++k)
                    if (ge[k] != 0.0) {
                        rowpos.push_back(k < 3 ? pg + k : pe + k - 3);
                        coef.push_back(ge[k]);
                    }
            }
            col_off[a * 12 + c + 1] = int32_t(rowpos.size());
            mom[size_t(a) * 12 + c] = 0.0;
        }
    }
    // LDS column -> stream position and weight kind of k_far_lambda (columns in the order
    // the kernel forms them, padded to whole batches)
    const int ncol = lam_ncol(p);
    std::vector<int32_t> cpos(size_t((ncol + LAM_TBL_MAX - 1) / LAM_TBL_MAX) * LAM_TBL_MAX, 0), ckind(cpos.size(), 0);
    for (int n = 0; n <= p + 1; ++n)
        for (int k3 = 0; k3 <= n; ++k3)
            for (int k2 = 0; k2 <= n - k3; ++k2) {
                const int q[3] = {n - k3 - k2, k2, k3};
                int pg, pe;
                stream_pos(p, q, pg, pe);
                cpos[lam_gcol(p, q[0], q[1], q[2])] = pg;
            }
    for (int n = 1; n <= p + 2; ++n) {
        const int ord = n - 1, base = ord > 0 ? nidx(ord - 1) : 0;
        for (int a = 0; a < n * (n + 1) / 2; ++a) {
            int q[3], pg, pe;
            kof(base + a, q);
            stream_pos(p, q, pg, pe);
            cpos[lam_ebase(p, n) + a] = pe;
            ckind[lam_ebase(p, n) + a] = 1;
        }
    }
    auto *t = new PhiT();
    t->p = p;
    auto up = [](DBuf &d, const void *src, size_t bytes) {
        d.reserve(bytes);
        if (bytes) STK_HIP(hipMemcpy(d.p, src, bytes, hipMemcpyHostToDevice));
    };
    up(t->col_off, col_off.data(), sizeof(int32_t) * col_off.size());
    up(t->rowpos, rowpos.data(), sizeof(int32_t) * rowpos.size());
    up(t->coef, coef.data(), sizeof(double) * coef.size());
    up(t->epow, epow.data(), sizeof(int32_t) * epow.size());
    up(t->cpos, cpos.data(), sizeof(int32_t) * cpos.size());
    up(t->ckind, ckind.data(), sizeof(int32_t) * ckind.size());
    g_phit[key] = t;
    return *t;
}

// lm[(node * nm + a) * 12 + c] = sum_pos S[pos, (a,c)] rho^-epow[pos] lambda[node][pos]
__global__ __launch_bounds__(256) void k_phi_adj(const double *__restrict__ lambda, const double *__restrict__ rho,
                                                 int nm, int ng, const int32_t *__restrict__ col_off,
                                                 const int32_t *__restrict__ rowpos, const double *__restrict__ coef,
                                                 const int32_t *__restrict__ epow, double *__restrict__ lm) {
    const int32_t node = blockIdx.x;
    const double inv = 1.0 / rho[node];
    const double *L = lambda + size_t(node) * 6 * ng;
    for (int col = threadIdx.x; col < 12 * nm; col += 256) {
        double s = 0.0;
        for (int e = col_off[col]; e < col_off[col + 1]; ++e) {
            const int pos = rowpos[e];
            double sc = 1.0;
            for (int k = 0; k < epow[pos]; ++k) sc *= inv;
            s += coef[e] * sc * L[pos];
        }
        lm[size_t(node) * nm * 12 + col] = s;
    }
}

// ---- totals, back to caller order --------------------------------------------------------
__global__ void k_src_total(const double *__restrict__ part, int nlev, int64_t n, const double *__restrict__ near,
                            const int32_t *__restrict__ perm, double *__restrict__ gf, double *__restrict__ gh,
                            double *__restrict__ gy) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double v[9];
    for (int q = 0; q < 9; ++q) v[q] = near[9 * j + q];
    for (int l = 0; l < nlev; ++l)
        for (int q = 0; q < 9; ++q) v[q] += part[(size_t(l) * n + j) * 9 + q];
    const int64_t o = perm[j];
    for (int q = 0; q < 3; ++q) {
        if (gf) gf[3 * o + q] = v[q];
        if (gh) gh[3 * o + q] = v[3 + q];
        if (gy) gy[3 * o + q] = v[6 + q];
    }
}

__global__ void k_tgt_total(const double *__restrict__ far, const double *__restrict__ near, int64_t m,
                            const int32_t *__restrict__ tperm, double *__restrict__ gt) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t o = tperm[t];
    for (int q = 0; q < 3; ++q) gt[3 * o + q] = far[3 * t + q] + near[3 * t + q];
}

__global__ void k_gather_w(const double *__restrict__ w, const int32_t *__restrict__ tperm, int64_t m,
                           double *__restrict__ ws) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= m) return;
    const int64_t o = tperm[t];
    for (int q = 0; q < 3; ++q) ws[3 * t + q] = w[3 * o + q];
}

template <typename T> void dispatch_adj(int p, const LambdaArgs &la, const TgradArgs &ta, hipStream_t s) {
    switch (p) {
#define STK_ADJ_CASE(P)                  \
    case P:                              \
        launch_far_lambda<P, T>(la, s);  \
        launch_far_tgrad<P, T>(ta, s);   \
        break;
        STK_ADJ_CASE(0)
        STK_ADJ_CASE(1)
        STK_ADJ_CASE(2)
        STK_ADJ_CASE(3)
        STK_ADJ_CASE(4)
        STK_ADJ_CASE(5)
        STK_ADJ_CASE(6)
        STK_ADJ_CASE(7)
        STK_ADJ_CASE(8)
        STK_ADJ_CASE(9)
        STK_ADJ_CASE(10)
#undef STK_ADJ_CASE
        default: throw Error(STK_EINVAL, "p out of range");
    }
}

void dispatch_src_grad(int p, const SrcGradArgs &a, int32_t nitems, hipStream_t s) {
    switch (p) {
        case 0: launch_src_grad<0>(a, nitems, s); break;
        case 1: launch_src_grad<1>(a, nitems, s); break;
        case 2: launch_src_grad<2>(a, nitems, s); break;
        case 3: launch_src_grad<3>(a, nitems, s); break;
        case 4: launch_src_grad<4>(a, nitems, s); break;
        case 5: launch_src_grad<5>(a, nitems, s); break;
        case 6: launch_src_grad<6>(a, nitems, s); break;
        case 7: launch_src_grad<7>(a, nitems, s); break;
        case 8: launch_src_grad<8>(a, nitems, s); break;
        case 9: launch_src_grad<9>(a, nitems, s); break;
        case 10: launch_src_grad<10>(a, nitems, s); break;
        default: throw Error(STK_EINVAL, "p out of range");
    }
}

// leaf-side work items: leaves that appear in some near list, in blocks of `per` points
__global__ void k_leaf_units(const int32_t *__restrict__ eoff, const int32_t *__restrict__ count, int32_t nn,
                             int32_t per, int32_t *__restrict__ cnt) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    cnt[c] = eoff[c + 1] > eoff[c] ? (count[c] + per - 1) / per : 0;
}

__global__ void k_leaf_fill(const int32_t *__restrict__ eoff, const int32_t *__restrict__ start,
                            const int32_t *__restrict__ count, const int32_t *__restrict__ ioff, int32_t nn, int32_t per,
                            int32_t *__restrict__ inode, int32_t *__restrict__ ia) {
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn || eoff[c + 1] == eoff[c]) return;
    int32_t it = ioff[c];
    for (int32_t b = 0; b < count[c]; b += per, ++it) {
        inode[it] = c;
        ia[it] = start[c] + b;
    }
}

// Re-sort group-major list entries by node: ent = entry positions ordered by node,
// ent_off = per-node offsets into ent, ent_group = entry -> group, plus work items
// (leaf, first point): blocks of per points of the leaves that have entries.
void transpose(Tree &t, const DBuf &goff, const DBuf &gnode, int64_t ne, int32_t ngroups, TransposedLists &tr,
               int32_t per, hipStream_t s) {
    const int32_t nn = t.nnodes;
    int32_t *eg = reserve<int32_t>(tr.ent_group, size_t(ne) + 1);
    hipLaunchKernelGGL(k_entry_group, dim3(nblk(ngroups, 256)), dim3(256), 0, s, goff.as<int32_t>(), ngroups, eg);
    STK_CHECK_LAUNCH();
    uint64_t *keys = reserve<uint64_t>(t.s_keys, size_t(ne) + 1);
    int32_t *ent = reserve<int32_t>(tr.ent, size_t(ne) + 1);
    if (ne > 0) {
        hipLaunchKernelGGL(k_node_keys, dim3(nblk(ne, 256)), dim3(256), 0, s, gnode.as<int32_t>(), ne, keys, ent);
        STK_CHECK_LAUNCH();
        int bits = 1;
        while ((int64_t(1) << bits) <= nn) ++bits;
        radix_sort_pairs(t, keys, ent, ne, bits, s);
    }
    int32_t *eoff = reserve<int32_t>(tr.ent_off, size_t(nn) + 1);
    hipLaunchKernelGGL(k_node_off, dim3(nblk(nn + 1, 256)), dim3(256), 0, s, keys, ne, nn, eoff);
    STK_CHECK_LAUNCH();
    int32_t *cnt = reserve<int32_t>(t.s_vals, size_t(nn) + 1);
    int32_t *ioff = reserve<int32_t>(t.s_vals2, size_t(nn) + 1);
    hipLaunchKernelGGL(k_leaf_units, dim3(nblk(nn, 256)), dim3(256), 0, s, eoff, t.ncount.as<int32_t>(), nn, per, cnt);
    STK_CHECK_LAUNCH();
    scan_exclusive_i32(cnt, ioff, nn, t.s_scan, s);
    int32_t nitems = 0;
    {
        const PeekSrc src{ioff + nn, 4};
        int64_t v = 0;
        peek(t.peek, s, 1, &src, &v);
        nitems = int32_t(v);
    }
    tr.nitems = nitems;
    int32_t *inode = reserve<int32_t>(tr.item_node, size_t(nitems) + 1);
    int32_t *ia = reserve<int32_t>(tr.item_a, size_t(nitems) + 1);
    hipLaunchKernelGGL(k_leaf_fill, dim3(nblk(nn, 256)), dim3(256), 0, s, eoff, t.nstart.as<int32_t>(),
                       t.ncount.as<int32_t>(), ioff, nn, per, inode, ia);
    STK_CHECK_LAUNCH();
}

}  // namespace

void adjoint(Plan &pl, const double *w, double *gf, double *gh, double *gt, double *gy, hipStream_t s) {
    Tree &t = *pl.tree;
    if (!t.have_moments) throw Error(STK_ESTATE, "the plan's tree has no moments");
    require(t.k_rhs == 1, "the adjoint supports one right-hand side");
    const int p = t.p, nm = nidx(p), ngc = nidx(p + 1);
    const int64_t m = pl.m, n = t.n;
    const int32_t nn = t.nnodes, ng = pl.ngroups;
    const bool src = gf || gh || gy;
    const bool fp64 = t.prec == STK_FP64;
    AdjScratch &A = pl.adj;
    prof_mark(-1, s);

    double *ws = reserve<double>(A.ws, size_t(m) * 3);
    hipLaunchKernelGGL(k_gather_w, dim3(nblk(m, 256)), dim3(256), 0, s, w, pl.tperm_p, m, ws);
    STK_CHECK_LAUNCH();

    NearAdjArgs na{};
    na.tpos = pl.tpos_p;
    na.ws = ws;
    na.m = m;
    na.off = pl.near_off.as<int32_t>();
    na.node = pl.near_node.as<int32_t>();
    na.mask = pl.near_mask.as<uint64_t>();
    na.start = t.nstart.as<int32_t>();
    na.count = t.ncount.as<int32_t>();
    na.geo = t.geo.as<double>();
    na.wts = t.wts.p;

    // target side
    double *gtn = nullptr, *gtf = nullptr;
    if (gt) {
        gtn = reserve<double>(A.gt_near, size_t(m) * 3);
        gtf = reserve<double>(A.gt_far, size_t(m) * 3);
        na.gt = gtn;
        NearTgradArgs nt{pl.tpos_p, ws, pl.ncm.item_node.as<int32_t>(), pl.ncm.item_i0.as<int32_t>(),
                         pl.ncm.item_i1.as<int32_t>(), pl.ncm.inc_tgt.as<int32_t>(), pl.ncm.inc_slot.as<int32_t>(),
                         t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), t.geo.as<double>(), t.wts.p,
                         pl.ncm.part.p, pl.ncm.n_items};
        const int32_t *toff = pl.ncm.toff.as<int32_t>();
        if (fp64) {
            if (nt.nitems > 0) {
                hipLaunchKernelGGL(k_near_tgrad<double>, dim3(xcd_item_blocks<XCD_CHUNK_NEAR>(nt.nitems)), dim3(64), 0, s, nt);
                STK_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_slot_reduce<double>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const double *>(nt.part), toff, m, gtn);
        } else {
            if (nt.nitems > 0) {
                hipLaunchKernelGGL(k_near_tgrad<float>, dim3(xcd_item_blocks<XCD_CHUNK_NEAR>(nt.nitems)), dim3(64), 0, s, nt);
                STK_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_slot_reduce<float>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const float *>(nt.part), toff, m, gtn);
        }
        STK_CHECK_LAUNCH();
    }

    // far field: stream adjoints (source side) and target gradients, both over the
    // cluster-major view of every far entry (64 incidences of one cluster per pass)
    LambdaArgs la{};
    TgradArgs ta{};
    PhiT &ph = phit_for(t.device, p);
    // (the forward's own view when it took every far entry cluster major)
    const bool reuse = pl.far_sparse_max >= 64;
    if ((src || gt) && pl.n_far_inc >= CM_MAX_INC)
        throw Error(STK_EINVAL, "adjoint: too many far interactions for the cluster-major lists");
    ClusterMajor &fc = reuse ? pl.fcm : A.far_cm;
    if ((src || gt) && !reuse)
        cluster_major(t, fc, pl.far_off.as<int32_t>(), pl.far_node.as<int32_t>(), pl.far_mask.as<uint64_t>(),
                      pl.n_far_entries, ng, m, 64, pl.cnt_far.as<int32_t>(), s);
    if (src) {
        // work items: runs of up to LAMBDA_RUN incidences of one cluster
        const int32_t *loff = fc.loff.as<int32_t>();
        int32_t *cnt = reserve<int32_t>(t.s_vals, size_t(nn) + 1);
        int32_t *ioff = reserve<int32_t>(t.s_vals2, size_t(nn) + 1);
        hipLaunchKernelGGL(k_item_count, dim3(nblk(nn, 256)), dim3(256), 0, s, loff, nn, LAMBDA_RUN, cnt);
        STK_CHECK_LAUNCH();
        scan_exclusive_i32(cnt, ioff, nn, t.s_scan, s);
        int32_t nitems = 0;
        {
            const PeekSrc src{ioff + nn, 4};
            int64_t v = 0;
            peek(t.peek, s, 1, &src, &v);
            nitems = int32_t(v);
        }
        TransposedLists &tr = A.far_t;
        tr.nitems = nitems;
        int32_t *inode = reserve<int32_t>(tr.item_node, size_t(nitems) + 1);
        int32_t *ia = reserve<int32_t>(tr.item_a, size_t(nitems) + 1);
        int32_t *ib = reserve<int32_t>(tr.item_b, size_t(nitems) + 1);
        if (nitems > 0) {
            hipLaunchKernelGGL(k_item_fill, dim3(nblk(nitems, 256)), dim3(256), 0, s, loff, ioff, nn, LAMBDA_RUN,
                               nitems, inode, ia, ib);
            STK_CHECK_LAUNCH();
        }
        double *lam = reserve<double>(A.lambda, size_t(nn) * 6 * ngc);
        STK_HIP(hipMemsetAsync(lam, 0, sizeof(double) * size_t(nn) * 6 * ngc, s));
        la.tpos = pl.tpos_p;
        la.ws = ws;
        la.m = m;
        la.item_node = inode;
        la.item_i0 = ia;
        la.item_i1 = ib;
        la.inc_tgt = fc.inc_tgt.as<int32_t>();
        la.center = t.ncenter.as<double>();
        la.rho = t.nrho.as<double>();
        la.cpos = ph.cpos.as<int32_t>();
        la.ckind = ph.ckind.as<int32_t>();
        la.lambda = lam;
        la.nitems = nitems;
    }
    if (gt) {
        const size_t tsz = fp64 ? sizeof(double) : sizeof(float);
        ta.tpos = pl.tpos_p;
        ta.ws = ws;
        ta.item_node = fc.item_node.as<int32_t>();
        ta.item_i0 = fc.item_i0.as<int32_t>();
        ta.item_i1 = fc.item_i1.as<int32_t>();
        ta.inc_tgt = fc.inc_tgt.as<int32_t>();
        ta.inc_slot = fc.inc_slot.as<int32_t>();
        ta.center = t.ncenter.as<double>();
        ta.rho = t.nrho.as<double>();
        ta.wblk = t.wblk.p;
        ta.part = reserve<unsigned char>(fc.part, tsz * 3 * size_t(fc.n_inc) + tsz);
        ta.nitems = fc.n_items;
    }
    if (fp64)
        dispatch_adj<double>(p, la, ta, s);
    else
        dispatch_adj<float>(p, la, ta, s);
    if (gt) {
        // each target's far terms added in the order of its own list
        const int32_t *toff = fc.toff.as<int32_t>();
        if (fp64)
            hipLaunchKernelGGL(k_slot_reduce<double>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const double *>(ta.part), toff, m, gtf);
        else
            hipLaunchKernelGGL(k_slot_reduce<float>, dim3(nblk(m, 256)), dim3(256), 0, s,
                               static_cast<const float *>(ta.part), toff, m, gtf);
        STK_CHECK_LAUNCH();
    }

    if (src) {
        // stream adjoints -> moment adjoints -> per-level source gradients
        double *lm = reserve<double>(A.lm, size_t(nn) * nm * 12);
        hipLaunchKernelGGL(k_phi_adj, dim3(nn), dim3(256), 0, s, A.lambda.as<double>(), t.nrho.as<double>(), nm, ngc,
                           ph.col_off.as<int32_t>(), ph.rowpos.as<int32_t>(), ph.coef.as<double>(),
                           ph.epow.as<int32_t>(), lm);
        STK_CHECK_LAUNCH();
        const int nlev = t.nlevels;
        double *part = reserve<double>(A.part, size_t(nlev) * n * 9);
        STK_HIP(hipMemsetAsync(part, 0, sizeof(double) * size_t(nlev) * n * 9, s));
        SrcGradArgs sa{t.pos.as<double>(), t.geo.as<double>(), t.w12.as<double>(), t.ncenter.as<double>(), lm,
                       t.nstart.as<int32_t>(), t.ncount.as<int32_t>(), t.chunk_off.as<int32_t>(),
                       t.nlevel.as<int32_t>(), nn, n, part};
        dispatch_src_grad(p, sa, t.nchunks, s);

        // near field, source side
        transpose(t, pl.near_off, pl.near_node, pl.n_near_entries, ng, A.near_t, 64, s);
        double *gs = reserve<double>(A.gs, size_t(n) * 9);
        STK_HIP(hipMemsetAsync(gs, 0, sizeof(double) * size_t(n) * 9, s));
        na.item_node = A.near_t.item_node.as<int32_t>();
        na.item_j0 = A.near_t.item_a.as<int32_t>();
        na.ent = A.near_t.ent.as<int32_t>();
        na.ent_off = A.near_t.ent_off.as<int32_t>();
        na.ent_group = A.near_t.ent_group.as<int32_t>();
        na.gs = gs;
        na.nitems = A.near_t.nitems;
        if (na.nitems > 0) {
            if (fp64)
                hipLaunchKernelGGL(k_near_sgrad<double>, dim3(na.nitems), dim3(64 * SG_WAVES), 0, s, na);
            else
                hipLaunchKernelGGL(k_near_sgrad<float>, dim3(na.nitems), dim3(64 * SG_WAVES), 0, s, na);
            STK_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_src_total, dim3(nblk(n, 256)), dim3(256), 0, s, part, nlev, n, gs,
                           t.perm.as<int32_t>(), gf, gh, gy);
        STK_CHECK_LAUNCH();
    }
    if (gt) {
        hipLaunchKernelGGL(k_tgt_total, dim3(nblk(m, 256)), dim3(256), 0, s, gtf, gtn, m, pl.tperm_p, gt);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_ADJOINT, s);
}

}  // namespace stk
