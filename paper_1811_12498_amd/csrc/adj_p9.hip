// Far-field adjoint for Taylor order p = 9: cluster stream adjoints (both precisions) and
// the per-source gradients from the moment adjoints.
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_lambda<9, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<9, double>(const LambdaArgs &, hipStream_t);
template void launch_src_grad<9>(const SrcGradArgs &, int32_t, hipStream_t);
}  // namespace stk
