// Far-field kernel on the matrix cores for Taylor order p = 5 (FP32, several right-hand sides).
#include "far_mfma.hpp"

namespace stk {
template void launch_far_mfma<5>(const FarArgs &, DBuf &, int32_t, hipStream_t);
}  // namespace stk
