// Far-field kernels for Taylor order p = 9, one right-hand side per pass (both precisions), and its
// cluster-major kernel for sparse far entries.
#include "far_impl.hpp"

namespace stk {
template void launch_far<9, float, 1>(const FarArgs &, hipStream_t);
template void launch_far<9, double, 1>(const FarArgs &, hipStream_t);
template void launch_far_sparse<9, float, 1>(const FarSparseArgs &, hipStream_t);
template void launch_far_sparse<9, double, 1>(const FarSparseArgs &, hipStream_t);
}  // namespace stk
