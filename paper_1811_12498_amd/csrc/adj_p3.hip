// Far-field adjoint kernels for Taylor order p = 3 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<3, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<3, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<3, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<3, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
