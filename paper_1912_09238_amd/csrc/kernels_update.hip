// Flux-update and set-up kernels (update.hpp, setup.hpp) for M = 1, 3, 4.
#include <hip/hip_runtime.h>

#include "kernel_select.hpp"

namespace ipm {

template <int M>
UpdFn update_pick(int G) {
  switch (G) {
    case 16: return update_kernel<M, 16>;
    case 32: return update_kernel<M, 32>;
    case 64: return update_kernel<M, 64>;
  }
  return nullptr;
}

template <int M>
const void* update_batched_pick(int G) {
  switch (G) {
    case 16: return reinterpret_cast<const void*>(update_batched<M, 16>);
    case 32: return reinterpret_cast<const void*>(update_batched<M, 32>);
    case 64: return reinterpret_cast<const void*>(update_batched<M, 64>);
  }
  return nullptr;
}

template <int M>
SetupFn setup_pick() {
  return setup_kernel<M>;
}

template UpdFn update_pick<1>(int);
template UpdFn update_pick<3>(int);
template UpdFn update_pick<4>(int);
template const void* update_batched_pick<1>(int);
template const void* update_batched_pick<3>(int);
template const void* update_batched_pick<4>(int);
template SetupFn setup_pick<1>();
template SetupFn setup_pick<3>();
template SetupFn setup_pick<4>();

}  // namespace ipm
