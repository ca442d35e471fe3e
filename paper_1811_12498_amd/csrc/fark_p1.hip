// Far-field kernels for Taylor order p = 1, FP32, 2 and 4 right-hand sides per pass (group and cluster major).
#include "far_impl.hpp"

namespace stk {
template void launch_far<1, float, 2>(const FarArgs &, hipStream_t);
template void launch_far<1, float, 4>(const FarArgs &, hipStream_t);
template void launch_far_sparse<1, float, 2>(const FarSparseArgs &, hipStream_t);
template void launch_far_sparse<1, float, 4>(const FarSparseArgs &, hipStream_t);
}  // namespace stk
