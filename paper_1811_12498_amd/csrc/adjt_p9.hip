// Far-field adjoint: target-position gradients for Taylor order p = 9 (both precisions).
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_tgrad<9, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<9, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
