// Regularized far-field kernel: cluster-major items (one cluster and up to 64 of the
// targets that accepted it), one lane per (target, cluster) interaction, evaluating the
// one-function form of reg_math.hpp against the cluster's stream.
#pragma once

#include "far_kernels.hpp"

namespace stk {

struct RegFarArgs {
    const double *tpos;                        // (m,3) sorted targets
    const int32_t *item_node, *item_i0, *item_i1;
    const int32_t *inc_tgt, *inc_slot;
    const double *center;                      // (nn,3)
    const double *wreg;                        // (nn, reg_stream_len(p)): each cluster's stream
    double *part;                              // (incidences, 3): each incidence's velocity at its slot
    double eps2;
    int32_t nitems;
};

// defined in reg_far_impl.hpp, instantiated per Taylor order in regf_p*.hip
template <int P> void launch_reg_far(const RegFarArgs &a, hipStream_t s);

}  // namespace stk
