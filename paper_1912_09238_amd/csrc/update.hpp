// Kinetic flux and moment update (Sec. 3.1 eq:momentIterationFunction in
// the quadrature form eq:momentUpQuadrature; Sec. 3.2), the time step, the
// steady residual eq:residualSteady and the per-step bookkeeping.
//
// A group of G lanes owns one cell.  Lanes over quadrature nodes read the
// nodal ansatz of the cell and its neighbours (written by the dual kernel),
// apply the deterministic numerical flux per node and form the nodal
// update u - dt/dx (g_r - g_l) [- dt/dy (g_n - g_s)] in LDS; lanes over
// moments then project it on the basis.  The old-moment term is the ansatz
// h(lambda_c) itself, as in eq:momentIterationFunction.  The last block to
// finish closes the step: time, residual (fixed summation order), done flag.
#pragma once

#include "dual_small.hpp"

namespace ipm {

struct UpdateParams {
  const double* __restrict__ wphi;   // [Q][kp]
  int N, Q, kp, cells, nx, ny, dim;
  const int8_t* __restrict__ cellN;
  const double* __restrict__ nodal;  // [cells][Q][M]
  const double* __restrict__ ghost;  // [4][Q][M] Dirichlet ghost nodal states
  const double* __restrict__ uold;   // [cells][M][N]
  double* __restrict__ unew;         // [cells][M][N]
  double* __restrict__ res_part;     // [gridDim.x]
  int bc[4];
  int flux;
  double gamma, cfl, dx, dy, vol, t_end, steady_eps;
  StepCtrl* ctrl;
  int parity;
};

template <int M>
__device__ __forceinline__ const double* neighbour_nodal(const UpdateParams& P, int ix, int iy,
                                                         int side) {
  int jx = ix, jy = iy;
  if (side == 0) --jx;
  if (side == 1) ++jx;
  if (side == 2) --jy;
  if (side == 3) ++jy;
  if (jx < 0 || jx >= P.nx || jy < 0 || jy >= P.ny) {
    const int bc = P.bc[side];
    if (bc == kBcPeriodic) {
      jx = (jx + P.nx) % P.nx;
      jy = (jy + P.ny) % P.ny;
    } else if (bc == kBcDirichlet) {
      return P.ghost + static_cast<size_t>(side) * P.Q * M;
    } else {
      jx = ix;
      jy = iy;
    }
  }
  return P.nodal + (static_cast<size_t>(jy) * P.nx + jx) * P.Q * M;
}

template <int M, int G>
__global__ __launch_bounds__(256) void update_kernel(UpdateParams P) {
  StepCtrl* C = P.ctrl;
  if (C->done) return;
  extern __shared__ double smem[];
  const int Q = P.Q, kp = P.kp, N = P.N;
  double* wphiL = smem;
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) wphiL[k] = P.wphi[k];
  constexpr int CPW = 64 / G;
  const int groups = (blockDim.x >> 6) * CPW;
  double* UT = wphiL + Q * kp;  // per group [Q][M]
  double* red = UT + static_cast<size_t>(groups) * Q * M;
  __shared__ int s_last;

  // time step from the largest wave speed of this step's ansatz (all cells,
  // all nodes, Dirichlet ghosts)
  double ax = C->ghost_amax[0], ay = C->ghost_amax[1];
  for (int s = 0; s < 64; ++s) {
    ax = nan_max(ax, __longlong_as_double(static_cast<long long>(C->amax[P.parity][0][s])));
    if (P.dim == 2)
      ay = nan_max(ay, __longlong_as_double(static_cast<long long>(C->amax[P.parity][1][s])));
  }
  const double t0 = C->t[P.parity];
  double dt = P.dim == 2 ? P.cfl / (ax / P.dx + ay / P.dy) : P.cfl * P.dx / ax;
  bool last = false;
  if (P.t_end > 0.0 && t0 + dt >= P.t_end) {
    dt = P.t_end - t0;
    last = true;
  }
  const double lfx = P.dx / (2.0 * dt), lfy = P.dy / (2.0 * dt);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int gid = (threadIdx.x >> 6) * CPW + lane / G;
  const int r = lane % G;
  const int cell = blockIdx.x * groups + gid;
  double* ut = UT + static_cast<size_t>(gid) * Q * M;
  double res_cell = 0.0;
  int finite = 1;
  if (cell < P.cells) {
    const int ix = cell % P.nx, iy = cell / P.nx;
    const double* uc = P.nodal + static_cast<size_t>(cell) * Q * M;
    const double* uw = neighbour_nodal<M>(P, ix, iy, 0);
    const double* ue = neighbour_nodal<M>(P, ix, iy, 1);
    const double* us = P.dim == 2 ? neighbour_nodal<M>(P, ix, iy, 2) : uc;
    const double* un = P.dim == 2 ? neighbour_nodal<M>(P, ix, iy, 3) : uc;
    const double rx = dt / P.dx, ry = dt / P.dy;
    for (int q = r; q < Q; q += G) {
      double c[M], l[M], rr[M], gl[M], gr[M], acc[M];
#pragma unroll
      for (int a = 0; a < M; ++a) {
        c[a] = uc[q * M + a];
        l[a] = uw[q * M + a];
        rr[a] = ue[q * M + a];
      }
      numerical_flux<M>(P.flux, P.gamma, 0, c, rr, lfx, gr);
      numerical_flux<M>(P.flux, P.gamma, 0, l, c, lfx, gl);
#pragma unroll
      for (int a = 0; a < M; ++a) acc[a] = c[a] - rx * (gr[a] - gl[a]);
      if (P.dim == 2) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
          l[a] = us[q * M + a];
          rr[a] = un[q * M + a];
        }
        numerical_flux<M>(P.flux, P.gamma, 1, c, rr, lfy, gr);
        numerical_flux<M>(P.flux, P.gamma, 1, l, c, lfy, gl);
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] -= ry * (gr[a] - gl[a]);
      }
#pragma unroll
      for (int a = 0; a < M; ++a) ut[q * M + a] = acc[a];
    }
    wave_sync();
    const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
    double d2 = 0.0;
    for (int k = r; k < M * N; k += G) {
      const int a = k / N, i = k % N;
      double s = 0.0;
      if (i < Nc)
        for (int q = 0; q < Q; ++q) s = fma(ut[q * M + a], wphiL[q * kp + i], s);
      const size_t off = static_cast<size_t>(cell) * M * N + k;
      const double d = s - P.uold[off];
      d2 = fma(d, d, d2);
      finite &= (s == s && fabs(s) < 1e300) ? 1 : 0;
      P.unew[off] = s;
    }
    d2 = group_sum<G>(d2);
    res_cell = P.vol * sqrt(d2);
  }
  finite = group_and<G>(finite);
  // fixed-order block partial of the residual
  if (r == 0) {
    red[2 * gid] = res_cell;
    red[2 * gid + 1] = finite ? 0.0 : 1.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, bad = 0.0;
    for (int k = 0; k < groups; ++k) {
      s += red[2 * k];
      bad += red[2 * k + 1];
    }
    P.res_part[blockIdx.x] = s;
    if (bad > 0.0 || !(ax == ax) || !(ay == ay) || !(dt > 0.0 || last)) atomicOr(&C->status, kStNonfinite);
    __threadfence();
    const unsigned prev = atomicAdd(&C->blocks_done, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // last block: residual in fixed order, then close the step
  const volatile double* rp = P.res_part;
  double s = 0.0;
  for (int k = threadIdx.x; k < static_cast<int>(gridDim.x); k += blockDim.x) s += rp[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double residual = red[0];
    C->t[P.parity ^ 1] = last ? P.t_end : t0 + dt;
    C->dt_last = dt;
    C->residual = residual;
    C->amax_last = P.dim == 2 ? nan_max(ax, ay) : ax;
    C->steps += 1;
    for (int k = 0; k < 64; ++k) {
      C->amax[P.parity ^ 1][0][k] = 0ull;
      C->amax[P.parity ^ 1][1][k] = 0ull;
    }
    C->blocks_done = 0u;
    const unsigned st = atomicOr(&C->status, 0u);
    if (last || (P.steady_eps > 0.0 && residual <= P.steady_eps) || st != 0u) C->done = 1;
  }
}

}  // namespace ipm
