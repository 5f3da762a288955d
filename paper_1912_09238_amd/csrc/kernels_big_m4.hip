// Workgroup-per-cell Newton kernels for M = 4.
#include <hip/hip_runtime.h>

#include "kernels_big.hpp"

namespace ipm {
template DualFn big_pick<4>(int, int);
template const void* big_batched_pick<4>(int, int);
}  // namespace ipm
