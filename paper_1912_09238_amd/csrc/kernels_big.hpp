// Workgroup-per-cell Newton kernels (dual_big.hpp) of one variable count M
// (1 or 4); included by one unit per M.
#pragma once

#include "chord_big.hpp"
#include "dual_big.hpp"
#include "kernel_select.hpp"

namespace ipm {

// prec bit 0: BF16-split MFMA Hessian (T >= 5); bit 1: inexact-Hessian
// Newton (any T: T < 5 serves small-cell classes with many nodes)
template <int M, int PR>
DualFn big_prec_pick(int T) {
  switch (T) {
    case 5: return newton_big_kernel<M, 5, PR>;
    case 6: return newton_big_kernel<M, 6, PR>;
    case 8: return newton_big_kernel<M, 8, PR>;
    case 9: return newton_big_kernel<M, 9, PR>;
  }
  if constexpr (PR == 2) switch (T) {
      case 1: return newton_big_kernel<M, 1, 2>;
      case 2: return newton_big_kernel<M, 2, 2>;
      case 4: return newton_big_kernel<M, 4, 2>;
    }
  return nullptr;
}

template <int M>
DualFn big_pick(int T, int prec) {
  if (prec == 10) switch (T) {  // the chord steps alone (chord_big.hpp)
      case 1: return newton_chord_big_kernel<M, 1>;
      case 2: return newton_chord_big_kernel<M, 2>;
      case 4: return newton_chord_big_kernel<M, 4>;
      case 5: return newton_chord_big_kernel<M, 5>;
      case 6: return newton_chord_big_kernel<M, 6>;
      case 8: return newton_chord_big_kernel<M, 8>;
      case 9: return newton_chord_big_kernel<M, 9>;
    }
  switch (prec) {
    case 1: return big_prec_pick<M, 1>(T);
    case 2: return big_prec_pick<M, 2>(T);
    case 3: return big_prec_pick<M, 3>(T);
  }
  switch (T) {
    case 1: return newton_big_kernel<M, 1>;
    case 2: return newton_big_kernel<M, 2>;
    case 4: return newton_big_kernel<M, 4>;
    case 5: return newton_big_kernel<M, 5>;
    case 6: return newton_big_kernel<M, 6>;
    case 8: return newton_big_kernel<M, 8>;
    case 9: return newton_big_kernel<M, 9>;
  }
  return nullptr;
}

template <int M, int PR>
const void* big_batched_prec_pick(int T) {
  switch (T) {
    case 5: return reinterpret_cast<const void*>(newton_big_batched<M, 5, PR>);
    case 6: return reinterpret_cast<const void*>(newton_big_batched<M, 6, PR>);
    case 8: return reinterpret_cast<const void*>(newton_big_batched<M, 8, PR>);
    case 9: return reinterpret_cast<const void*>(newton_big_batched<M, 9, PR>);
  }
  if constexpr (PR == 2) switch (T) {
      case 1: return reinterpret_cast<const void*>(newton_big_batched<M, 1, 2>);
      case 2: return reinterpret_cast<const void*>(newton_big_batched<M, 2, 2>);
      case 4: return reinterpret_cast<const void*>(newton_big_batched<M, 4, 2>);
    }
  return nullptr;
}

template <int M>
const void* big_batched_pick(int T, int prec) {
  if (prec == 10) switch (T) {
      case 1: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 1>);
      case 2: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 2>);
      case 4: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 4>);
      case 5: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 5>);
      case 6: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 6>);
      case 8: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 8>);
      case 9: return reinterpret_cast<const void*>(newton_chord_big_batched<M, 9>);
    }
  switch (prec) {
    case 1: return big_batched_prec_pick<M, 1>(T);
    case 2: return big_batched_prec_pick<M, 2>(T);
    case 3: return big_batched_prec_pick<M, 3>(T);
  }
  switch (T) {
    case 1: return reinterpret_cast<const void*>(newton_big_batched<M, 1>);
    case 2: return reinterpret_cast<const void*>(newton_big_batched<M, 2>);
    case 4: return reinterpret_cast<const void*>(newton_big_batched<M, 4>);
    case 5: return reinterpret_cast<const void*>(newton_big_batched<M, 5>);
    case 6: return reinterpret_cast<const void*>(newton_big_batched<M, 6>);
    case 8: return reinterpret_cast<const void*>(newton_big_batched<M, 8>);
    case 9: return reinterpret_cast<const void*>(newton_big_batched<M, 9>);
  }
  return nullptr;
}

}  // namespace ipm
