// Kernel selection across translation units.  Every kernel template is
// instantiated in exactly one unit (kernels_dual_m*.hip, kernels_big_m*.hip,
// kernels_update.hip), so the units compile in parallel and no kernel is
// registered twice; the host runtime reaches them through these functions.
#pragma once

#include "dual.hpp"
#include "setup.hpp"
#include "update.hpp"

namespace ipm {

using DualFn = void (*)(DualParams);
using UpdFn = void (*)(UpdateParams);
using SetupFn = void (*)(SetupParams);

// register-row Newton kernel of NP lanes per cell (prec 0: exact; 2:
// inexact-Hessian; 10: the inexact-Hessian chord steps alone), single
// problem and batched; null when not built
template <int M> DualFn dual_pick(int NP, int prec);
template <int M> const void* dual_batched_pick(int NP, int prec);
// workgroup-per-cell Newton kernel with T x T tiles (prec bit 0: BF16 MFMA
// Hessian, T >= 5; bit 1: inexact-Hessian; 10: its chord steps alone, one
// cell per wavefront); M = 1 or 4
template <int M> DualFn big_pick(int T, int prec);
template <int M> const void* big_batched_pick(int T, int prec);
// flux update with G lanes per cell, and the set-up kernel
template <int M> UpdFn update_pick(int G);
template <int M> const void* update_batched_pick(int G);
template <int M> SetupFn setup_pick();

extern template DualFn dual_pick<1>(int, int);
extern template DualFn dual_pick<3>(int, int);
extern template DualFn dual_pick<4>(int, int);
extern template const void* dual_batched_pick<1>(int, int);
extern template const void* dual_batched_pick<3>(int, int);
extern template const void* dual_batched_pick<4>(int, int);
extern template DualFn big_pick<1>(int, int);
extern template DualFn big_pick<4>(int, int);
extern template const void* big_batched_pick<1>(int, int);
extern template const void* big_batched_pick<4>(int, int);
extern template UpdFn update_pick<1>(int);
extern template UpdFn update_pick<3>(int);
extern template UpdFn update_pick<4>(int);
extern template const void* update_batched_pick<1>(int);
extern template const void* update_batched_pick<3>(int);
extern template const void* update_batched_pick<4>(int);
extern template SetupFn setup_pick<1>();
extern template SetupFn setup_pick<3>();
extern template SetupFn setup_pick<4>();

}  // namespace ipm
