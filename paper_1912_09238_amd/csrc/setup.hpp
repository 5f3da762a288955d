// Initial state (Alg. 1, first loop): cell-average moments
// uhat_j^0 = <u_IC(x_j, .) phi>_Q from nodal values at the cell centre, and
// the starting dual lambda^0 = <grad s(u_IC(x_j, .)) phi>_Q (the projection
// of the entropy variables), which the dual kernel then converges.
#pragma once

#include "device_common.hpp"

namespace ipm {

struct SetupParams {
  const double* __restrict__ wphi;   // [Q][kp]
  int N, Q, kp, cells;
  const int8_t* __restrict__ cellN;
  const double* __restrict__ ic_nodal;    // [cells][Q][M] or null
  const double* __restrict__ ic_moments;  // [cells][M][N] (if ic_nodal is null)
  const double* __restrict__ ic_dual;     // [cells][M][N] or null
  double* __restrict__ uhat;
  double* __restrict__ lam;
  ClosureParams cp;
  unsigned* status;
};

// one thread per (cell, moment) entry, layout [cell][M][N]
template <int M>
__global__ __launch_bounds__(256) void setup_kernel(SetupParams P) {
  const size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t total = static_cast<size_t>(P.cells) * M * P.N;
  if (k >= total) return;
  const int cell = static_cast<int>(k / (static_cast<size_t>(M) * P.N));
  const int a = static_cast<int>((k / P.N) % M);
  const int i = static_cast<int>(k % P.N);
  const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : P.N;
  if (i >= Nc) {
    P.uhat[k] = 0.0;
    P.lam[k] = 0.0;
    return;
  }
  bool ok = true;
  double u_i = 0.0, l_i = 0.0;
  if (P.ic_nodal) {
    const double* nod = P.ic_nodal + static_cast<size_t>(cell) * P.Q * M;
    for (int q = 0; q < P.Q; ++q) {
      const double wf = P.wphi[q * P.kp + i];
      double L[M];
      ok &= entropy_gradient<M>(P.cp, nod + q * M, L);
      u_i = fma(nod[q * M + a], wf, u_i);
      l_i = fma(L[a], wf, l_i);
    }
  } else {
    // moments given: start from the entropy variables of the mean state
    const double* mom = P.ic_moments + static_cast<size_t>(cell) * M * P.N;
    double mean[M], L[M];
#pragma unroll
    for (int b = 0; b < M; ++b) mean[b] = mom[b * P.N];
    ok = entropy_gradient<M>(P.cp, mean, L);
    u_i = mom[a * P.N + i];
    l_i = (i == 0) ? L[a] : 0.0;
  }
  if (P.ic_dual) {
    l_i = P.ic_dual[k];
    ok = true;
  }
  P.uhat[k] = u_i;
  P.lam[k] = l_i;
  if (!ok) atomicOr(P.status, kStRealizability);
}

}  // namespace ipm
