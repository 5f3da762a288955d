// Fused per-cell dual solve for n = m*N <= 64 unknowns (Sec. 3.1: eq:L,
// eq:dualIterationFunction, eq:tauCrit; one-shot: eq:oneshotIPMdual).
//
// Layout: a group of NP lanes (NP = 8/16/32/64, the smallest >= n) owns
// one cell, 64/NP cells per wavefront.  Unknowns are interleaved,
// r = i*m + a (mode i, conserved variable a), so every lower-degree basis is
// a prefix and register indices stay compile-time constants.
//   - ansatz evaluation: lanes over quadrature nodes; u_s and the packed
//     Jacobian grad u_s go to LDS;
//   - gradient and the tau test: lanes over unknowns, FP64;
//   - Hessian: lane r accumulates its full row H[r][0..NP) in registers,
//     H[(i,a)][(k,b)] = sum_q w_q J_q[a][b] phi_i(xi_q) phi_k(xi_q);
//   - solve H d = g by Gauss-Jordan elimination without pivoting (H is
//     SPD): at step k the pivot row equals the pivot column of the
//     symmetric Schur complement, so one LDS column broadcast per step
//     feeds every row, the right-hand side is eliminated alongside, and no
//     triangular back-substitution (no transposed access) is needed;
//   - Newton update with the backtracking rule on L (see DESIGN notes):
//     Armijo backtracking when the dual residual exceeds 1e-6, else t = 1;
//     one-shot: exactly one full step.
// The converged dual, the nodal ansatz values (read by the flux update) and
// the per-step statistics (Newton counts, largest wave speed) leave the
// kernel; the Hessian never touches HBM.
#pragma once

#include "device_common.hpp"

namespace ipm {

struct StepCtrl {
  double t[2];                        // time, double-buffered by step parity
  unsigned long long amax[2][2][64];  // [parity][direction][slot] speed bit patterns
  double ghost_amax[2];               // Dirichlet ghost speeds (x, y)
  unsigned long long newton_iters;
  unsigned long long steps;
  unsigned int max_iters;
  unsigned int status;
  unsigned int setup_status;
  unsigned int blocks_done;
  double dt_last, residual, amax_last;
  int done;
  int pad_;
};

struct DualParams {
  const double* __restrict__ phi;   // [Q][kp] Phi, zero padded to kp columns
  const double* __restrict__ wphi;  // [Q][kp] w_q Phi (column 0 holds w_q)
  int N, Q, kp, cells;
  const int8_t* __restrict__ cellN; // modes per cell, or null (all N)
  const double* __restrict__ uhat;  // [cells][M][N]
  double* __restrict__ lam;         // [cells][M][N], in/out
  double* __restrict__ nodal;       // [cells][Q][M], out
  ClosureParams cp;
  double tau;
  int max_newton, one_shot;
  int mode;                         // 0: time step (stats, speeds), 1: setup
  int dim;
  StepCtrl* ctrl;
  int parity;
};

template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// max that keeps NaN (a NaN wave speed must reach the time-step logic)
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a == a && b == b) ? fmax(a, b) : __longlong_as_double(0x7ff8000000000000LL);
}

template <int G>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, G));
  return v;
}

template <int G>
__device__ __forceinline__ int group_and(int v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v &= __shfl_xor(v, o, G);
  return v;
}

template <int M, int NP>
struct SmallDual {
  static constexpr int G = NP;
  static constexpr int CPW = 64 / NP;
  static constexpr int NJ = M * (M + 1) / 2;

  __host__ __device__ static int group_doubles(int Q) {
    return NP + Q * M + Q * NJ + 2 * (NP + 2) + NP;
  }
  __host__ __device__ static size_t lds_bytes(int Q, int kp, int waves) {
    return sizeof(double) * (2 * static_cast<size_t>(Q) * kp +
                             static_cast<size_t>(waves) * CPW * group_doubles(Q) +
                             static_cast<size_t>(waves) * CPW * 4);
  }

  // Ansatz at the trial dual lamS for the nodes of this lane.  Writes u and
  // packed J to LDS, returns the lane's share of <s_*> and the admissible flag.
  __device__ static int eval(const DualParams& P, const double* lamS, int Nc, const double* phiL,
                             const double* wphiL, int lane_r, double* US, double* JS,
                             double& ssum) {
    int ok = 1;
    ssum = 0.0;
    for (int q = lane_r; q < P.Q; q += G) {
      double L[M];
#pragma unroll
      for (int a = 0; a < M; ++a) L[a] = 0.0;
      const double* ph = phiL + q * P.kp;
      for (int i = 0; i < Nc; ++i) {
        const double f = ph[i];
#pragma unroll
        for (int a = 0; a < M; ++a) L[a] = fma(lamS[i * M + a], f, L[a]);
      }
      double u[M], J[NJ], ss;
      ok &= closure<M>(P.cp, L, u, J, ss) ? 1 : 0;
#pragma unroll
      for (int a = 0; a < M; ++a) US[q * M + a] = u[a];
#pragma unroll
      for (int k = 0; k < NJ; ++k) JS[q * NJ + k] = J[k];
      ssum = fma(wphiL[q * P.kp], ss, ssum);
    }
    return ok;
  }
};

template <int M, int NP>
__global__ __launch_bounds__(256) void dual_small_kernel(DualParams P) {
  using S = SmallDual<M, NP>;
  constexpr int G = S::G, CPW = S::CPW, NJ = S::NJ;
  if (P.mode == 0 && P.ctrl->done) return;

  extern __shared__ double smem[];
  const int Q = P.Q, kp = P.kp, N = P.N;
  double* phiL = smem;
  double* wphiL = phiL + Q * kp;
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) {
    phiL[k] = P.phi[k];
    wphiL[k] = P.wphi[k];
  }
  const int waves = blockDim.x >> 6;
  const int groups = waves * CPW;
  double* stats = wphiL + Q * kp + static_cast<size_t>(groups) * S::group_doubles(Q);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int gid = (threadIdx.x >> 6) * CPW + lane / G;
  const int r = lane % G;
  const int cell = blockIdx.x * groups + gid;
  double* lamS = wphiL + Q * kp + static_cast<size_t>(gid) * S::group_doubles(Q);
  double* US = lamS + NP;
  double* JS = US + Q * M;
  double* colA = JS + Q * NJ;
  double* colB = colA + NP + 2;
  double* gS = colB + NP + 2;

  int its = 0;
  unsigned status = 0;
  double sx = 0.0, sy = 0.0;

  if (cell < P.cells) {
    const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
    const int nc = Nc * M;
    const int i = r / M, a = r % M;
    const bool live = r < nc;
    const size_t base = static_cast<size_t>(cell) * M * N + static_cast<size_t>(a) * N + i;
    double lam_r = live ? P.lam[base] : 0.0;
    const double uh_r = live ? P.uhat[base] : 0.0;

    lamS[r] = lam_r;
    wave_sync();
    double ssum;
    int ok = group_and<G>(S::eval(P, lamS, Nc, phiL, wphiL, r, US, JS, ssum));
    wave_sync();

    auto gradient = [&](double& g_out) -> double {
      double g = 0.0;
      if (live) {
        for (int q = 0; q < Q; ++q) g = fma(US[q * M + a], wphiL[q * kp + i], g);
        g -= uh_r;
      }
      g_out = g;
      gS[r] = g * g;
      wave_sync();
      double res = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) {
        double s2 = 0.0;
        for (int k = 0; k < Nc; ++k) s2 += gS[k * M + b];
        res += sqrt(s2);
      }
      wave_sync();
      return res;
    };

    double g_r;
    double res = ok ? gradient(g_r) : 0.0;
    if (!ok) status |= kStRealizability;

    while (ok) {
      if (!(res == res) || res > 1e300) {
        status |= kStNonfinite;
        break;
      }
      if (!P.one_shot) {
        if (res < P.tau) break;
        if (its >= P.max_newton) {
          status |= kStNewton;
          break;
        }
      }
      // ---- Hessian rows in registers
      double row[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) row[c] = 0.0;
      const double live_f = live ? 1.0 : 0.0;
      for (int q = 0; q < Q; ++q) {
        const double wi = wphiL[q * kp + i] * live_f;
        const double* Jq = JS + q * NJ;
        double s[M];
#pragma unroll
        for (int b = 0; b < M; ++b) s[b] = Jq[Packed<M>::idx(a, b)] * wi;
        const double* ph = phiL + q * kp;
#pragma unroll
        for (int c = 0; c < NP; ++c) row[c] = fma(s[c % M], ph[c / M], row[c]);
      }
      // ---- Gauss-Jordan solve H d = g
      double x = g_r, diag = 1.0;
      int chol_ok = 1;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        if (k < nc) {
          double* cb = (k & 1) ? colB : colA;
          cb[r] = row[k];
          if (r == k) cb[NP] = x;
          wave_sync();
          const double piv = cb[k];
          const double gk = cb[NP];
          chol_ok &= piv > 0.0 ? 1 : 0;
          const double rp = 1.0 / piv;
          if (r == k) diag = piv;
          const double f = (r == k) ? 0.0 : row[k] * rp;
#pragma unroll
          for (int j = k + 1; j < NP; ++j) row[j] = fma(-f, cb[j], row[j]);
          x = fma(-f, gk, x);
        }
      }
      if (!chol_ok) {
        status |= kStCholesky;
        break;
      }
      const double d_r = live ? x / diag : 0.0;
      // ---- step length
      const bool ls = !P.one_shot && res > 1e-6;
      double L0 = 0.0, slope = 0.0;
      if (ls) {
        L0 = group_sum<G>(ssum) - group_sum<G>(lam_r * uh_r);
        slope = group_sum<G>(g_r * d_r);
      }
      double t = 1.0, lt_r = lam_r;
      int accepted = 0;
      for (int h = 0; h <= 60; ++h) {
        lt_r = lam_r - t * d_r;
        lamS[r] = lt_r;
        wave_sync();
        ok = group_and<G>(S::eval(P, lamS, Nc, phiL, wphiL, r, US, JS, ssum));
        wave_sync();
        if (!ls) {
          accepted = 1;
          break;
        }
        if (ok) {
          const double Lt = group_sum<G>(ssum) - group_sum<G>(lt_r * uh_r);
          if (Lt <= L0 - 1e-4 * t * slope) {
            accepted = 1;
            break;
          }
        }
        t *= 0.5;
      }
      if (!accepted) {
        status |= kStLineSearch;
        break;
      }
      lam_r = lt_r;
      ++its;
      if (!ok) {
        status |= kStRealizability;
        break;
      }
      res = gradient(g_r);
      if (P.one_shot) break;
    }

    // ---- write back: dual, nodal ansatz, wave speeds
    if (live) P.lam[base] = lam_r;
    for (int q = r; q < Q; q += G) {
      double u[M];
#pragma unroll
      for (int b = 0; b < M; ++b) u[b] = US[q * M + b];
#pragma unroll
      for (int b = 0; b < M; ++b) P.nodal[(static_cast<size_t>(cell) * Q + q) * M + b] = u[b];
      if (P.mode == 0) {
        double ax, ay;
        wave_speeds<M>(P.cp.gamma, P.dim, u, ax, ay);
        sx = nan_max(sx, ax);
        sy = nan_max(sy, ay);
      }
    }
  }

  // ---- block reduction of the statistics, one atomic per block
  if (P.mode == 0) {
    sx = group_max<G>(sx);
    sy = group_max<G>(sy);
  }
  if (r == 0) {
    stats[gid * 4 + 0] = static_cast<double>(its);
    stats[gid * 4 + 1] = static_cast<double>(status);
    stats[gid * 4 + 2] = sx;
    stats[gid * 4 + 3] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum_its = 0;
    unsigned max_its = 0, st = 0;
    double mx = 0.0, my = 0.0;
    const int live_groups = min(groups, P.cells - static_cast<int>(blockIdx.x) * groups);
    for (int k = 0; k < live_groups; ++k) {
      const unsigned it = static_cast<unsigned>(stats[k * 4 + 0]);
      sum_its += it;
      max_its = max(max_its, it);
      st |= static_cast<unsigned>(stats[k * 4 + 1]);
      const double ax = stats[k * 4 + 2], ay = stats[k * 4 + 3];
      mx = nan_max(mx, ax);
      my = nan_max(my, ay);
    }
    if (P.mode == 0) {
      atomicAdd(&P.ctrl->newton_iters, sum_its);
      atomicMax(&P.ctrl->max_iters, max_its);
      if (st) atomicOr(&P.ctrl->status, st);
      const int slot = blockIdx.x & 63;
      atomicMax(&P.ctrl->amax[P.parity][0][slot], speed_bits(mx));
      if (P.dim == 2) atomicMax(&P.ctrl->amax[P.parity][1][slot], speed_bits(my));
    } else if (st) {
      atomicOr(&P.ctrl->setup_status, st);
    }
  }
}

}  // namespace ipm
