// Far-field adjoint: target-position gradients for Taylor order p = 6 (both precisions).
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_tgrad<6, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<6, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
