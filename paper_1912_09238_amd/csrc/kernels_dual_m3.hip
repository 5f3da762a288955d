// Register-row Newton kernels for M = 3.
#include <hip/hip_runtime.h>

#include "kernels_dual.hpp"

namespace ipm {
template DualFn dual_pick<3>(int, int);
template const void* dual_batched_pick<3>(int, int);
}  // namespace ipm
