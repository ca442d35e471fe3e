// Far-field adjoint kernels for Taylor order p = 2 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<2, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<2, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<2, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<2, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
