// Far-field adjoint: target-position gradients for Taylor order p = 10 (both precisions).
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_tgrad<10, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<10, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
