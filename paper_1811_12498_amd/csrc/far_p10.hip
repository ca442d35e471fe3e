// Far-field kernels for Taylor order p = 10 (both precisions).
#include "far_kernels.hpp"

namespace stk {
template void launch_far<10, float>(const FarArgs &, hipStream_t);
template void launch_far<10, double>(const FarArgs &, hipStream_t);
}  // namespace stk
