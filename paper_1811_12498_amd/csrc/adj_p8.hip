// Far-field adjoint kernels for Taylor order p = 8 (both precisions).
#include "adjoint_far.hpp"

namespace stk {
template void launch_far_lambda<8, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<8, double>(const LambdaArgs &, hipStream_t);
template void launch_far_tgrad<8, float>(const TgradArgs &, hipStream_t);
template void launch_far_tgrad<8, double>(const TgradArgs &, hipStream_t);
}  // namespace stk
