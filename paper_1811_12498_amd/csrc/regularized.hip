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
// field runs k_near_reg on the leaf-major items.  The far field writes both kernels as
// derivatives of R (reg_math.hpp): u_i = sum_q a^q W_i^q over the Taylor coefficients a^q
// of R to order p + 3 and a stream W per cluster, which k_reg_stream builds from the
// moments; k_reg_far evaluates it on cluster-major items (every far entry transposed),
// one lane per (target, cluster) interaction.
#include "reg_far.hpp"
#include "reg_math.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

// grid (nnodes): each cluster's stream (reg_math.hpp), reg_stream_len(p) values per node,
// from the node's 12 nm moments staged in LDS (every moment feeds many stream values)
__global__ __launch_bounds__(64) void k_reg_stream(const double *__restrict__ mom, int p, int nm,
                                                   double *__restrict__ wreg) {
    extern __shared__ double ms[];  // [nm][12]
    const int32_t node = blockIdx.x;
    const double *src = mom + size_t(node) * nm * 12;
    for (int i = threadIdx.x; i < 12 * nm; i += 64) ms[i] = src[i];
    __syncthreads();
    double *out = wreg + size_t(node) * reg_stream_len(p);
    for (int a = nidx(1) + threadIdx.x; a < nidx(p + 3); a += 64)
        reg_stream_fill(ms, 12, p, a, out);
}

void dispatch_reg_far(int p, const RegFarArgs &a, hipStream_t s) {
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
    prof_mark(STK_PHASE_LISTS, s);  // the lists transposed
    double *part = reserve<double>(cm.part, 3 * size_t(cm.n_inc) + 1);
    double *wreg = reserve<double>(t.wreg, size_t(t.nnodes) * reg_stream_len(t.p));
    if (pl.moments_ready) {  // moments computed on another stream
        STK_HIP(hipStreamWaitEvent(s, pl.moments_ready, 0));
        pl.moments_ready = nullptr;
    }
    if (t.nnodes > 0) {
        hipLaunchKernelGGL(k_reg_stream, dim3(unsigned(t.nnodes)), dim3(64), sizeof(double) * 12 * nidx(t.p), s,
                           t.mom.as<double>(), t.p, nidx(t.p), wreg);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_MOMENTS, s);  // the clusters' streams, like the channel blocks
    RegFarArgs ra{pl.tpos_p, cm.item_node.as<int32_t>(), cm.item_i0.as<int32_t>(),
                  cm.item_i1.as<int32_t>(), cm.inc_tgt.as<int32_t>(), cm.inc_slot.as<int32_t>(),
                  t.ncenter.as<double>(), wreg, part, eps * eps, cm.n_items};
    dispatch_reg_far(t.p, ra, s);
    if (m > 0) {
        hipLaunchKernelGGL(k_reg_finish, dim3(unsigned((m + 255) / 256)), dim3(256), 0, s, part,
                           cm.toff.as<int32_t>(), unear, pl.tperm_p, m, u_out);
        STK_CHECK_LAUNCH();
    }
    prof_mark(STK_PHASE_FAR, s);
}

}  // namespace stk
