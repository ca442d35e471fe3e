// Far-field adjoint: target-position gradients for Taylor order p = 0 (both precisions).
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_tgrad<0, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<0, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
