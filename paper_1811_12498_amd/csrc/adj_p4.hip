// Far-field adjoint kernels for Taylor order p = 4 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<4, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<4, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<4, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<4, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
