// Register-row Newton kernels (dual.hpp) of one variable count M; included
// by one unit per M.
#pragma once

#include "chord.hpp"
#include "kernel_select.hpp"

namespace ipm {

// prec 0: exact Newton; 2: inexact-Hessian (full kernel); 10: its chord
// steps alone (chord.hpp); 4 and 6: 0 and 2 for rules of at most NP nodes
template <int M>
DualFn dual_pick(int NP, int prec) {
  if (prec == 10) switch (NP) {
      case 8: return newton_chord_kernel<M, 8>;
      case 16: return newton_chord_kernel<M, 16>;
      case 32: return newton_chord_kernel<M, 32>;
      case 64: return newton_chord_kernel<M, 64>;
    }
  if (prec == 2) switch (NP) {
      case 8: return newton_kernel<M, 8, 2>;
      case 16: return newton_kernel<M, 16, 2>;
      case 32: return newton_kernel<M, 32, 2>;
      case 64: return newton_kernel<M, 64, 2>;
    }
  if (prec == 4 || prec == 6) {
    if (prec == 4) switch (NP) {
        case 8: return newton_kernel<M, 8, 4>;
        case 16: return newton_kernel<M, 16, 4>;
        case 32: return newton_kernel<M, 32, 4>;
        case 64: return newton_kernel<M, 64, 4>;
      }
    switch (NP) {
      case 8: return newton_kernel<M, 8, 6>;
      case 16: return newton_kernel<M, 16, 6>;
      case 32: return newton_kernel<M, 32, 6>;
      case 64: return newton_kernel<M, 64, 6>;
    }
    return nullptr;
  }
  if (prec != 0) return nullptr;
  switch (NP) {
    case 8: return newton_kernel<M, 8>;
    case 16: return newton_kernel<M, 16>;
    case 32: return newton_kernel<M, 32>;
    case 64: return newton_kernel<M, 64>;
  }
  return nullptr;
}

template <int M>
const void* dual_batched_pick(int NP, int prec) {
  if (prec == 10) switch (NP) {
      case 8: return reinterpret_cast<const void*>(newton_chord_batched<M, 8>);
      case 16: return reinterpret_cast<const void*>(newton_chord_batched<M, 16>);
      case 32: return reinterpret_cast<const void*>(newton_chord_batched<M, 32>);
      case 64: return reinterpret_cast<const void*>(newton_chord_batched<M, 64>);
    }
  if (prec == 2) switch (NP) {
      case 8: return reinterpret_cast<const void*>(newton_batched<M, 8, 2>);
      case 16: return reinterpret_cast<const void*>(newton_batched<M, 16, 2>);
      case 32: return reinterpret_cast<const void*>(newton_batched<M, 32, 2>);
      case 64: return reinterpret_cast<const void*>(newton_batched<M, 64, 2>);
    }
  if (prec == 4 || prec == 6) {
    if (prec == 4) switch (NP) {
        case 8: return reinterpret_cast<const void*>(newton_batched<M, 8, 4>);
        case 16: return reinterpret_cast<const void*>(newton_batched<M, 16, 4>);
        case 32: return reinterpret_cast<const void*>(newton_batched<M, 32, 4>);
        case 64: return reinterpret_cast<const void*>(newton_batched<M, 64, 4>);
      }
    switch (NP) {
      case 8: return reinterpret_cast<const void*>(newton_batched<M, 8, 6>);
      case 16: return reinterpret_cast<const void*>(newton_batched<M, 16, 6>);
      case 32: return reinterpret_cast<const void*>(newton_batched<M, 32, 6>);
      case 64: return reinterpret_cast<const void*>(newton_batched<M, 64, 6>);
    }
    return nullptr;
  }
  if (prec != 0) return nullptr;
  switch (NP) {
    case 8: return reinterpret_cast<const void*>(newton_batched<M, 8>);
    case 16: return reinterpret_cast<const void*>(newton_batched<M, 16>);
    case 32: return reinterpret_cast<const void*>(newton_batched<M, 32>);
    case 64: return reinterpret_cast<const void*>(newton_batched<M, 64>);
  }
  return nullptr;
}

}  // namespace ipm
