// Regularized far-field kernel for Taylor order p = 2.
#include "reg_far_impl.hpp"

namespace stk {
template void launch_reg_far<2>(const RegFarArgs &, hipStream_t);
}  // namespace stk
