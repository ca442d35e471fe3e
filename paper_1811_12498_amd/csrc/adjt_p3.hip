// Far-field adjoint: target-position gradients for Taylor order p = 3 (both precisions).
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_tgrad<3, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<3, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
