// Far-field kernels for Taylor order p = 1 (both precisions).
#include "far_kernels.hpp"

namespace stk {
template void launch_far<1, float>(const FarArgs &, hipStream_t);
template void launch_far<1, double>(const FarArgs &, hipStream_t);
}  // namespace stk
