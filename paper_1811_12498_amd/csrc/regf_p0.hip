// Regularized far-field kernel for Taylor order p = 0.
#include "reg_far_impl.hpp"

namespace stk {
template void launch_reg_far<0>(const RegFarArgs &, hipStream_t);
}  // namespace stk
