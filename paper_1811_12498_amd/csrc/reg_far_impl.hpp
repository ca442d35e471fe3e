// Regularized far-field kernel body (instantiated per Taylor order in regf_p*.hip).
#pragma once

#include "reg_far.hpp"
#include "reg_math.hpp"

namespace stk {

// Workgroups of REG_WPB waves, wave w of block b on cluster-major item REG_WPB b + w:
// consecutive items mostly share their cluster, and the waves of one workgroup share a CU
// and its scalar cache, so one fetch of a stream line serves them all.  Each lane
// evaluates its target's interaction with the item's cluster (the stream is wave-uniform:
// scalar loads, SGPR operands) and writes the velocity to the interaction's slot in its
// target's list.
constexpr int32_t REG_WPB = 4;
template <int P> __global__ __launch_bounds__(64 * REG_WPB) void k_reg_far(RegFarArgs a) {
    using Eval = RegEval<P, true>;
    const int32_t it = xcd_item<XCD_CHUNK_FAR / REG_WPB>() * REG_WPB + int32_t(threadIdx.x >> 6);
    if (it >= a.nitems) return;
    const int lane = threadIdx.x & 63;
    const int32_t c = __builtin_amdgcn_readfirstlane(a.item_node[it]);
    const int32_t i0 = a.item_i0[it];
    if (lane < a.item_i1[it] - i0) {
        const int64_t t = a.inc_tgt[i0 + lane];
        const int32_t slot = a.inc_slot[i0 + lane];
        const double d[3] = {a.tpos[3 * t] - a.center[3 * c], a.tpos[3 * t + 1] - a.center[3 * c + 1],
                             a.tpos[3 * t + 2] - a.center[3 * c + 2]};
        const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + a.eps2;
        double u[3];
        Eval::run(d, R2, (typename Eval::Ptr)(a.wreg + size_t(c) * Eval::WS), u);
        double *o = a.part + 3 * int64_t(slot);
        o[0] = u[0];
        o[1] = u[1];
        o[2] = u[2];
    }
}

template <int P> void launch_reg_far(const RegFarArgs &a, hipStream_t s) {
    if (a.nitems == 0) return;
    const int32_t blocks = (a.nitems + REG_WPB - 1) / REG_WPB;
    hipLaunchKernelGGL(k_reg_far<P>, dim3(xcd_item_blocks<XCD_CHUNK_FAR / REG_WPB>(blocks)), dim3(64 * REG_WPB), 0,
                       s, a);
    STK_CHECK_LAUNCH();
}

}  // namespace stk
