// Far-field kernel on the matrix cores for Taylor order p = 7 (FP32, several right-hand sides).
#include "far_mfma.hpp"

namespace stk {
template void launch_far_mfma<7>(const FarArgs &, DBuf &, int32_t, hipStream_t);
}  // namespace stk
