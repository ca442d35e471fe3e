// Far-field adjoint for Taylor order p = 6: cluster stream adjoints (both precisions) and
// the per-source gradients from the moment adjoints.
#include "adjoint_far_impl.hpp"

namespace stk {
template void launch_far_lambda<6, float>(const LambdaArgs &, hipStream_t);
template void launch_far_lambda<6, double>(const LambdaArgs &, hipStream_t);
template void launch_src_grad<6>(const SrcGradArgs &, int32_t, hipStream_t);
}  // namespace stk
