// Register-row Newton kernels for M = 4.
#include <hip/hip_runtime.h>

#include "kernels_dual.hpp"

namespace ipm {
template DualFn dual_pick<4>(int, int);
template const void* dual_batched_pick<4>(int, int);
}  // namespace ipm
