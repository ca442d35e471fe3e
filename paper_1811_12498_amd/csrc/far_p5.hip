// Far-field kernels for Taylor order p = 5 (both precisions).
#include "far_kernels.hpp"

namespace stk {
template void launch_far<5, float>(const FarArgs &, hipStream_t);
template void launch_far<5, double>(const FarArgs &, hipStream_t);
}  // namespace stk
