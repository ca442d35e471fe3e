// Regularized Stokeslets and stresslets: the treecode with the kernels of the method of
// regularized Stokeslets (the extension Sec. 7 names as future work), FP64, one
// right-hand side.  R^2 = |d|^2 + eps^2:
//   S^eps_ij  = delta_ij (|d|^2 + 2 eps^2) / R^3 + d_i d_j / R^3,
//   T^eps_ijl = [d_i d_j d_l + (eps^2/2)(delta_ij d_l + delta_jl d_i + delta_il d_j)] / R^5
// (the regularized Stokeslet of Cortez, Fauci and Medovikov 2005 and -1/6 of the stress of
// its flow, normalised like eqs. Stokeslet and stresslet, which they equal at eps = 0).
//
// The tree, the moments (they do not depend on the kernel), the target order and the
// interaction lists (eq. MAC, Algorithm 1) are those of the plain evaluation; the near
// field runs k_near_reg on the leaf-major items, the far field k_reg_far_cm on
// cluster-major items (every far entry transposed).  The far field expands the kernels in y
// about the cluster centre to order p, u_i = sum_k a^k_ij M_j^k + at^k_ijl Mt_jl^k, with
// the coefficients built from the Taylor coefficients g_nu^k of R^(-2 nu), nu = 1/2, 3/2,
// 5/2, which follow recurrence_1 generalised to R^2 = |d|^2 + eps^2 and exponent nu,
//   n R^2 g^k = (2n + 2nu - 2) sum_i d_i g^(k-e_i) - (n + 2nu - 2) sum_i g^(k-2e_i),
// and the product rule on the linear factors d = x - y (each y-derivative of a factor d_i
// gives -e_i):
//   a^k_ij   = delta_ij (b^k + eps^2 c^k) + d_i d_j c^k - d_i c^(k-e_j) - d_j c^(k-e_i) + c^(k-e_i-e_j)
//   at^k_ijl = d_i d_j d_l e^k - d_j d_l e^(k-e_i) - d_i d_l e^(k-e_j) - d_i d_j e^(k-e_l)
//              + d_l e^(k-e_i-e_j) + d_j e^(k-e_i-e_l) + d_i e^(k-e_j-e_l) - e^(k-e_i-e_j-e_l)
//              + (eps^2/2)[delta_ij (d_l e^k - e^(k-e_l)) + delta_jl (d_i e^k - e^(k-e_i))
//                          + delta_il (d_j e^k - e^(k-e_j))]
// with b, c, e the coefficients for nu = 1/2, 3/2, 5/2 (terms with a negative index vanish).
#include "far_kernels.hpp"
#include "stk_internal.hpp"
#include "stk_math.hpp"

namespace stk {
namespace {

// Positions of the shifted multi-indices, per multi-index k (graded-lex position q):
// slots 0..2 hold k - e_i, slots 3..8 k - e_i - e_j (i <= j), slots 9..18
// k - e_i - e_j - e_l (i <= j <= l); -1 where a component is negative.
constexpr int TSLOTS = 19;
__host__ __device__ constexpr int pslot(int i, int j) {  // i, j in any order
    const int a = i < j ? i : j, b = i < j ? j : i;
    return 3 + (a == 0 ? b : (a == 1 ? 2 + b : 5));
}
__host__ __device__ constexpr int tslot(int i, int j, int l) {  // i, j, l in any order
    int a = i, b = j, c = l, x = 0;
    if (a > b) { x = a; a = b; b = x; }
    if (b > c) { x = b; b = c; c = x; }
    if (a > b) { x = a; a = b; b = x; }
    // 000 001 002 011 012 022 111 112 122 222
    return 9 + (a == 0 ? (b == 0 ? c : (b == 1 ? 2 + c : 5)) : (a == 1 ? (b == 1 ? 5 + c : 8) : 9));
}

// coefficient of family f at table entry `slot` of the current multi-index
template <int NM>
__device__ inline double gat(const double (&gl)[3][NM], int f, const int16_t *row, int slot) {
    const int a = row[slot];
    return a < 0 ? 0.0 : gl[f][a];
}

struct RegCmArgs {
    const double *tpos;      // (m,3) sorted targets
    const int32_t *item_node, *item_i0, *item_i1;
    const int32_t *inc_tgt, *inc_slot;
    const double *center;    // (nn,3)
    const double *mom;       // (nn, nm, 12): M_j (0..2), Mt_jl (3 + 3j + l)
    double *part;            // (incidences, 3): each incidence's velocity at its slot
    double eps2;
    int32_t nitems;
};

// One wave per cluster-major item (one cluster and up to 64 of the targets that accept it).
// The wave evaluates the item's interactions one after another: for each, its lanes build
// the three coefficient families order by order in LDS (the multi-indices of one order
// spread over the lanes), every lane contracts its share of the multi-indices with the
// cluster's moments (read from global memory, L1-resident after the first interaction)
// and a butterfly sum over the wave gives the velocity, which the target's lane writes to
// its incidence's slot; k_cm_add later adds the slots of each target in list order.
template <int P> __global__ __launch_bounds__(64) void k_reg_far_cm(RegCmArgs a) {
    constexpr int NM = nidx(P);
    __shared__ double gl[3][NM];
    __shared__ int16_t tab[NM][TSLOTS];
    const int32_t it = xcd_item<XCD_CHUNK_FAR>();
    if (it >= a.nitems) return;
    const int lane = threadIdx.x;
    for (int q = lane; q < NM; q += 64) {
        const int k1 = kof1c(q), k2 = kof2c(q), k3 = ordc(q) - k1 - k2;
        const int k[3] = {k1, k2, k3};
        for (int i = 0; i < 3; ++i) {
            int m1[3] = {k[0], k[1], k[2]};
            --m1[i];
            tab[q][i] = int16_t(gidx(m1[0], m1[1], m1[2]));
            for (int j = i; j < 3; ++j) {
                int m2[3] = {m1[0], m1[1], m1[2]};
                --m2[j];
                tab[q][pslot(i, j)] = int16_t(gidx(m2[0], m2[1], m2[2]));
                for (int l = j; l < 3; ++l) {
                    int m3[3] = {m2[0], m2[1], m2[2]};
                    --m3[l];
                    tab[q][tslot(i, j, l)] = int16_t(gidx(m3[0], m3[1], m3[2]));
                }
            }
        }
    }
    const int32_t c = __builtin_amdgcn_readfirstlane(a.item_node[it]);
    const int32_t i0 = a.item_i0[it];
    const int32_t nt = __builtin_amdgcn_readfirstlane(a.item_i1[it] - i0);
    const bool on = lane < nt;
    int32_t slot = 0;
    double x0 = 0, x1 = 0, x2 = 0;
    if (on) {
        const int64_t t = a.inc_tgt[i0 + lane];
        slot = a.inc_slot[i0 + lane];
        x0 = a.tpos[3 * t];
        x1 = a.tpos[3 * t + 1];
        x2 = a.tpos[3 * t + 2];
    }
    const double yc0 = a.center[3 * c], yc1 = a.center[3 * c + 1], yc2 = a.center[3 * c + 2];
    const double *__restrict__ mc = a.mom + size_t(c) * NM * 12;
    const double e2 = a.eps2;
    double mine[3] = {0.0, 0.0, 0.0};
    for (int bt = 0; bt < nt; ++bt) {
        const double d[3] = {__shfl(x0, bt) - yc0, __shfl(x1, bt) - yc1, __shfl(x2, bt) - yc2};
        const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + e2;
        const double ri = 1.0 / sqrt(R2);
        __syncthreads();  // the table is built / the previous interaction is done with gl
        if (lane == 0) {
            gl[0][0] = ri;
            gl[1][0] = ri * ri * ri;
            gl[2][0] = ri * ri * ri * ri * ri;
        }
        __syncthreads();
        for (int n = 1; n <= P; ++n) {
            const int cnt = (n + 1) * (n + 2) / 2, base = nidx(n - 1);
            const double inv = 1.0 / (double(n) * R2);
            for (int j = lane; j < cnt; j += 64) {
                const int q = base + j;
                const int16_t *row = tab[q];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int nu2 = 2 * f + 1;
                    double s1 = 0.0, s2 = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        s1 += d[i] * gat<NM>(gl, f, row, i);
                        s2 += gat<NM>(gl, f, row, pslot(i, i));
                    }
                    gl[f][q] = (double(2 * n + nu2 - 2) * s1 - double(n + nu2 - 2) * s2) * inv;
                }
            }
            __syncthreads();
        }
        // Contraction, with the sums over j, l taken against the moments first:
        //   sum_j a_ij M_j  = (b + eps^2 c) M_i + d_i (d.M) c - d_i sum_j c_(-j) M_j
        //                     - (d.M) c_(-i) + sum_j c_(-i-j) M_j
        //   sum_jl at_ijl Mt_jl = (d_i e - e_(-i)) Q - d_i (S1 + S2 - S3)
        //                     + sum_j e_(-i-j) (Mtd_j + dMt_j) - sum_jl e_(-i-j-l) Mt_jl
        //                     + (eps^2/2)[e (Mtd_i + dMt_i) - sum_l e_(-l) (Mt_il + Mt_li)
        //                                 + (d_i e - e_(-i)) tr]
        // with Q = d.Mt.d, Mtd = Mt d, dMt = d Mt, tr = trace Mt, S1 = e_(-j).Mtd,
        // S2 = e_(-l).dMt, S3 = sum_jl e_(-j-l) Mt_jl (c_(-i) = c^(k - e_i), and so on).
        double v[3] = {0.0, 0.0, 0.0};
        for (int q = lane; q < NM; q += 64) {
            const int16_t *row = tab[q];
            const double bk = gl[0][q], ck = gl[1][q], ek = gl[2][q];
            const double *Mq = mc + 12 * q;
            const double M[3] = {Mq[0], Mq[1], Mq[2]};
            double Mt[3][3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int l = 0; l < 3; ++l) Mt[j][l] = Mq[3 + 3 * j + l];
            double cm[3], em[3], Mtd[3], dMt[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                cm[i] = gat<NM>(gl, 1, row, i);
                em[i] = gat<NM>(gl, 2, row, i);
                Mtd[i] = Mt[i][0] * d[0] + Mt[i][1] * d[1] + Mt[i][2] * d[2];
                dMt[i] = d[0] * Mt[0][i] + d[1] * Mt[1][i] + d[2] * Mt[2][i];
            }
            const double dM = d[0] * M[0] + d[1] * M[1] + d[2] * M[2];
            const double cM = cm[0] * M[0] + cm[1] * M[1] + cm[2] * M[2];
            const double Q = d[0] * Mtd[0] + d[1] * Mtd[1] + d[2] * Mtd[2];
            const double tr = Mt[0][0] + Mt[1][1] + Mt[2][2];
            const double S1 = em[0] * Mtd[0] + em[1] * Mtd[1] + em[2] * Mtd[2];
            const double S2 = em[0] * dMt[0] + em[1] * dMt[1] + em[2] * dMt[2];
            double S3 = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int l = 0; l < 3; ++l) S3 += gat<NM>(gl, 2, row, pslot(j, l)) * Mt[j][l];
#pragma unroll 1
            for (int i = 0; i < 3; ++i) {
                double vs = (bk + e2 * ck) * M[i] + d[i] * dM * ck - d[i] * cM - dM * cm[i];
                double vt = (d[i] * ek - em[i]) * Q - d[i] * (S1 + S2 - S3);
                double e3 = 0.0, xs = 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    vs += gat<NM>(gl, 1, row, pslot(i, j)) * M[j];
                    vt += gat<NM>(gl, 2, row, pslot(i, j)) * (Mtd[j] + dMt[j]);
                    xs += em[j] * (Mt[i][j] + Mt[j][i]);
#pragma unroll
                    for (int l = 0; l < 3; ++l) e3 += gat<NM>(gl, 2, row, tslot(i, j, l)) * Mt[j][l];
                }
                vt += -e3 + 0.5 * e2 * (ek * (Mtd[i] + dMt[i]) - xs + (d[i] * ek - em[i]) * tr);
                v[i] += vs + vt;
            }
        }
        // butterfly sum over the wave: every lane ends with the same total
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            v[0] += __shfl_xor(v[0], o);
            v[1] += __shfl_xor(v[1], o);
            v[2] += __shfl_xor(v[2], o);
        }
        if (lane == bt) {
            mine[0] = v[0];
            mine[1] = v[1];
            mine[2] = v[2];
        }
    }
    if (on) {
        double *o = a.part + int64_t(slot) * 3;
        o[0] = mine[0];
        o[1] = mine[1];
        o[2] = mine[2];
    }
}

template <int P> void launch_reg_far(const RegCmArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    hipLaunchKernelGGL(k_reg_far_cm<P>, dim3(xcd_item_blocks<XCD_CHUNK_FAR>(a.nitems)), dim3(64), 0, s, a);
    STK_CHECK_LAUNCH();
}

void dispatch_reg_far(int p, const RegCmArgs &a, hipStream_t s) {
    switch (p) {
    case 0: launch_reg_far<0>(a, s); break;
    case 1: launch_reg_far<1>(a, s); break;
    case 2: launch_reg_far<2>(a, s); break;
    case 3: launch_reg_far<3>(a, s); break;
    case 4: launch_reg_far<4>(a, s); break;
    case 5: launch_reg_far<5>(a, s); break;
    case 6: launch_reg_far<6>(a, s); break;
    case 7: launch_reg_far<7>(a, s); break;
    case 8: launch_reg_far<8>(a, s); break;
    case 9: launch_reg_far<9>(a, s); break;
    case 10: launch_reg_far<10>(a, s); break;
    default: throw Error(STK_EINVAL, "p out of range");
    }
}

// per (target, right-hand side): far velocities in list order (compensated) plus the near
// part, written in the caller's order
__global__ void k_reg_finish(const double *__restrict__ part, const int32_t *__restrict__ toff,
                             const double *__restrict__ unear, const int32_t *__restrict__ tperm, int64_t m,
                             double *__restrict__ u_out) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= m) return;
    Comp<double> acc[3];
    for (int32_t k = toff[t]; k < toff[t + 1]; ++k)
        for (int q = 0; q < 3; ++q) acc[q].add(part[3 * int64_t(k) + q]);
    const int64_t o = tperm[t];
    for (int q = 0; q < 3; ++q) u_out[3 * o + q] = acc[q].value() + unear[3 * t + q];
}

}  // namespace

void evaluate_regularized(Tree &t, Plan &pl, const double *tgt, int64_t m, double theta, double eps,
                          double *u_out, bool same_as_sources, hipStream_t s) {
    require(t.have_moments && t.prec == STK_FP64 && t.k_rhs == 1,
            "regularized evaluation: the tree needs FP64 moments of one right-hand side");
    build_lists(t, pl, tgt, m, theta, same_as_sources, s);
    pl.reg_eps = eps;
    pl.far_sparse_max = 64;
    double *unear = reserve<double>(t.s_tmp, size_t(m) * 3);
    near_field(t, pl, unear, s);
    // every far entry cluster major: items of one cluster and up to 64 targets
    if (pl.n_far_inc >= CM_MAX_INC)
        throw Error(STK_EINVAL, "too many far-field (target, cluster) pairs for the cluster-major lists");
    ClusterMajor &cm = pl.fcm;
    cluster_major(t, cm, pl.far_off.as<int32_t>(), pl.far_node.as<int32_t>(), pl.far_mask.as<uint64_t>(),
                  pl.n_far_entries, pl.ngroups, m, 64, pl.cnt_far.as<int32_t>(), s);
    double *part = reserve<double>(cm.part, 3 * size_t(cm.n_inc) + 1);
    RegCmArgs ra{pl.tpos.as<double>(), cm.item_node.as<int32_t>(), cm.item_i0.as<int32_t>(),
                 cm.item_i1.as<int32_t>(), cm.inc_tgt.as<int32_t>(), cm.inc_slot.as<int32_t>(),
                 t.ncenter.as<double>(), t.mom.as<double>(), part, eps * eps, cm.n_items};
    dispatch_reg_far(t.p, ra, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_reg_finish, dim3(unsigned((m + 255) / 256)), dim3(256), 0, s, part,
                           cm.toff.as<int32_t>(), unear, pl.tperm.as<int32_t>(), m, u_out);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_FAR, s);
}

}  // namespace stk
