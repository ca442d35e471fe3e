// Far-field adjoint kernels for Taylor order p = 10 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<10, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<10, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<10, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<10, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
