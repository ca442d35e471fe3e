// Far-field adjoint kernels for Taylor order p = 6 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<6, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<6, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<6, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<6, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
