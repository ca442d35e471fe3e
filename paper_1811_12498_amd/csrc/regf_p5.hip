// Regularized far-field kernel for Taylor order p = 5.
#include "reg_far_impl.hpp"

namespace stk {
template void launch_reg_far<5>(const RegFarArgs &, hipStream_t);
}  // namespace stk
