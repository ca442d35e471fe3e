// Far-field kernels for Taylor order p = 8, one right-hand side per pass (both precisions), and its
// cluster-major kernel for sparse far entries.
#include "far_impl.hpp"

namespace stk {
template void launch_far<8, float, 1>(const FarArgs &, hipStream_t);
template void launch_far<8, double, 1>(const FarArgs &, hipStream_t);
template void launch_far_sparse<8, float, 1>(const FarSparseArgs &, hipStream_t);
template void launch_far_sparse<8, double, 1>(const FarSparseArgs &, hipStream_t);
}  // namespace stk
