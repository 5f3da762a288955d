// Register-row Newton kernels for M = 1.
#include <hip/hip_runtime.h>

#include "kernels_dual.hpp"

namespace ipm {
template DualFn dual_pick<1>(int, int);
template const void* dual_batched_pick<1>(int, int);
}  // namespace ipm
