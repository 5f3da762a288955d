// Workgroup-per-cell Newton kernels for M = 1.
#include <hip/hip_runtime.h>

#include "kernels_big.hpp"

namespace ipm {
template DualFn big_pick<1>(int, int);
template const void* big_batched_pick<1>(int, int);
}  // namespace ipm
