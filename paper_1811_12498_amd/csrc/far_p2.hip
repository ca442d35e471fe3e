// Far-field kernels for Taylor order p = 2 (both precisions).
#include "far_kernels.hpp"

namespace stk {
template void launch_far<2, float>(const FarArgs &, hipStream_t);
template void launch_far<2, double>(const FarArgs &, hipStream_t);
}  // namespace stk
