// Regularized far-field kernel for Taylor order p = 7.
#include "reg_far_impl.hpp"

namespace stk {
template void launch_reg_far<7>(const RegFarArgs &, hipStream_t);
}  // namespace stk
