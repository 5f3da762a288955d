// Per-cell dual solve (Sec. 3.1: eq:L, eq:dualIterationFunction,
// eq:tauCrit; one-shot: eq:oneshotIPMdual), n = m*N <= 64 unknowns.
//
// The tau test at the warm start of a time step is taken by the flux-update
// kernel of the previous step (it holds h(lambda) and the new moments), which
// lists the cells that need Newton steps in 64 lists; the other cells keep
// their dual and nodal ansatz unchanged, exactly as a solve that stops at
// iteration 0 would.
//  * newton_kernel: one wavefront per listed cell (or per cell in one-shot
//    and setup runs) iterates Newton to tau:
//      - unknowns interleaved r = i*m + a (mode i, variable a), so a lower
//        degree is a prefix;
//      - ansatz: lanes over nodes, u_s and the packed grad u_s to LDS;
//      - gradient and the tau test on sum_a |g_a|_2, FP64, reductions on
//        the DPP network;
//      - Hessian H[(i,a)][(k,b)] = sum_q w_q J_q[a][b] phi_i phi_k: lane r
//        accumulates row r in registers;
//      - H d = g: Gauss-Jordan elimination without pivoting (H is SPD).
//        Rows and columns beyond the cell's n unknowns are an identity
//        block, so every pivot step runs unconditionally.  At each step all
//        rows publish their entry in the pivot column through LDS; by
//        symmetry of the Schur complement this column is also the pivot row,
//        so every row is updated from it, the right-hand side is eliminated
//        along, and no back-substitution (no transposed access) is needed;
//      - step length: Armijo backtracking on L when the dual residual
//        exceeds 1e-6, else the full step; one-shot: one full step.
// The dual, the nodal ansatz (read by the flux update) and the wave speeds
// leave the kernels; the Hessian never touches HBM.  Statistics go to
// per-block cumulative counters (plain stores) and to 64 atomic speed slots
// on separate cache lines; no device-scope fence is issued.
#pragma once

#include "device_common.hpp"

namespace ipm {

constexpr int kSlots = 64;
constexpr int kSlotStride = 16;  // 128-byte spacing of atomic slots

struct StepCtrl {
  double t[2];                      // time by step parity
  int done[2];                      // stop flag by step parity
  unsigned int status;              // sticky failure bits
  unsigned int setup_status;
  unsigned long long steps;         // completed steps
  double ghost_amax[2];             // Dirichlet ghost speeds (x, y)
  double dt_last, residual, amax_last;
  unsigned long long newton_iters;  // filled by the close kernel
  unsigned int max_iters;
  unsigned int pad_;
  // [parity][direction][slot * kSlotStride] speed bit patterns
  unsigned long long amax[2][2][kSlots * kSlotStride];
  // [parity][slot * kSlotStride] lengths of the 64 lists of cells that
  // need Newton steps
  unsigned int list_len[2 * kSlots * kSlotStride];
};

struct DualParams {
  const double* __restrict__ phi;   // [Q][kp] Phi, zero padded to kp columns
  const double* __restrict__ wphi;  // [Q][kp] w_q Phi (column 0 holds w_q)
  int N, Q, kp, cells;
  const int8_t* __restrict__ cellN; // modes per cell, or null (all N)
  const double* __restrict__ uhat;  // [cells][M][N]
  double* __restrict__ lam;         // [cells][M][N], in/out
  double* __restrict__ nodal;       // [cells][Q][M], out
  unsigned long long* __restrict__ blk_stats;  // [gridDim.x][2]: iterations, max
  ClosureParams cp;
  double tau;
  int max_newton, one_shot;
  int mode;                         // 0: time step, 1: setup (converge only)
  int dim;
  StepCtrl* ctrl;
  int parity;
  int* __restrict__ lists;          // [64][list_cap] cells needing Newton steps (this step)
  int list_cap;                     // 0: newton_kernel takes cells in order
};

// ---------------------------------------------------------------- helpers

// max that keeps NaN (a NaN wave speed must reach the time-step logic)
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a == a && b == b) ? fmax(a, b) : __longlong_as_double(0x7ff8000000000000LL);
}

// Cross-lane traffic on the DPP network.  Row = 16 lanes.  quad_perm
// [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror = 0x141,
// row_mirror = 0x140, row_ror:8 = 0x128.  Reductions leave bitwise-identical
// results in every lane of the group (pairwise sums of the same operands,
// rows combined in a fixed order through readlane).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

template <int W>  // aligned groups of W = 1..16 lanes
__device__ __forceinline__ double lanes_sum(double v) {
  if (W >= 2) v += dpp_mov<0xB1>(v);
  if (W >= 4) v += dpp_mov<0x4E>(v);
  if (W >= 8) v += dpp_mov<0x141>(v);
  if (W >= 16) v += dpp_mov<0x140>(v);
  return v;
}

template <int G>  // aligned groups of G = 1..64 lanes
__device__ __forceinline__ double group_sum(double v) {
  if (G <= 16) return lanes_sum<G>(v);
  v = lanes_sum<16>(v);
  const double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16);
  const double r2 = readlane_d(v, 32), r3 = readlane_d(v, 48);
  if (G == 64) return (r0 + r1) + (r2 + r3);
  return ((threadIdx.x & 63) < 32) ? r0 + r1 : r2 + r3;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

__device__ __forceinline__ double wave_max(double v) {
  v = nan_max(v, dpp_mov<0xB1>(v));
  v = nan_max(v, dpp_mov<0x4E>(v));
  v = nan_max(v, dpp_mov<0x141>(v));
  v = nan_max(v, dpp_mov<0x140>(v));
  return nan_max(nan_max(readlane_d(v, 0), readlane_d(v, 16)),
                 nan_max(readlane_d(v, 32), readlane_d(v, 48)));
}

// every active lane's flag set
__device__ __forceinline__ int wave_all(int v) { return __ballot(!v) == 0ull ? 1 : 0; }

// value held by lane ^ X
template <int X>
__device__ __forceinline__ double xor_lane(double v) {
  if (X == 1) return dpp_mov<0xB1>(v);
  if (X == 2) return dpp_mov<0x4E>(v);
  if (X == 8) return dpp_mov<0x128>(v);
  return __shfl_xor(v, X, 64);
}

// 1/x: hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// Ansatz at the nodes q = q0, q0 + step, ... of one cell for the dual lamS
// (interleaved, first Nc modes).  Writes u and packed J to LDS, adds the
// lane's share of <s_*> to ssum.  Returns the admissible flag.
template <int M>
__device__ __forceinline__ int eval_nodes(const DualParams& P, const double* lamS, int Nc,
                                          const double* phiL, const double* wphiL, int q0,
                                          int step, double* US, double* JS, double& ssum) {
  constexpr int NJ = M * (M + 1) / 2;
  int ok = 1;
#pragma unroll 1
  for (int q = q0; q < P.Q; q += step) {
    double L[M];
#pragma unroll
    for (int a = 0; a < M; ++a) L[a] = 0.0;
    const double* ph = phiL + q * P.kp;
#pragma unroll 4
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

// ---------------------------------------------------------------- Newton

// Layout: a group of G = NP lanes owns one cell, 64/NP cells per wavefront,
// four wavefronts per block.  Lane r of a group holds row r of the Hessian
// (all NP columns) and the unknown r.  Control flow is uniform within a
// group; groups of one wavefront may leave the Newton loop at different
// iterations (all cross-lane operations stay inside the group).
template <int M, int NP>
struct NewtonCfg {
  static constexpr int G = NP;
  static constexpr int CPW = 64 / NP;
  static constexpr int NJ = M * (M + 1) / 2;
  static constexpr int KCOL = (NP + M - 1) / M;  // table columns the rows read

  __host__ __device__ static int group_doubles(int Q) {
    return NP + Q * (M + NJ) + 2 * NP + 2 + NP;
  }
  __host__ __device__ static size_t lds_bytes(int Q, int kp, int waves) {
    // tables, per-group work areas, then 2 stats per group + 2 speeds per wave
    return sizeof(double) * (2 * static_cast<size_t>(Q) * kp +
                             static_cast<size_t>(waves) * CPW * group_doubles(Q) +
                             2 * static_cast<size_t>(waves) * (CPW + 1));
  }
};

template <int M, int NP>
__global__ __launch_bounds__(256) void newton_kernel(DualParams P) {
  using Cfg = NewtonCfg<M, NP>;
  constexpr int G = Cfg::G, CPW = Cfg::CPW, NJ = Cfg::NJ;
  if (P.mode == 0 && (P.ctrl->done[P.parity] || P.ctrl->status)) return;
  if (P.mode == 0 && blockIdx.x == 0) {
    // the flux update of this step fills the next step's speed slots and list
    StepCtrl* C = P.ctrl;
    for (int k = threadIdx.x; k < kSlots; k += blockDim.x) {
      C->amax[P.parity ^ 1][0][k * kSlotStride] = 0ull;
      C->amax[P.parity ^ 1][1][k * kSlotStride] = 0ull;
      C->list_len[(P.parity ^ 1) * kSlots * kSlotStride + k * kSlotStride] = 0u;
    }
  }
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G;
  const int r = lane % G;
  // work item of this group: entry-major over the 64 lists, or the cell index
  const int item = (blockIdx.x * waves + wave) * CPW + grp;
  int cell = -1;
  if (P.list_cap > 0) {
    const int slot = item & (kSlots - 1), entry = item >> 6;
    const int len =
        static_cast<int>(P.ctrl->list_len[P.parity * kSlots * kSlotStride + slot * kSlotStride]);
    if (entry < min(len, P.list_cap)) cell = P.lists[static_cast<size_t>(slot) * P.list_cap + entry];
  } else if (item < P.cells) {
    cell = item;
  }
  if (!__syncthreads_or(cell >= 0)) return;

  const int Q = P.Q, kp = P.kp, N = P.N;
  extern __shared__ double smem[];
  double* phiL = smem;
  double* wphiL = phiL + Q * kp;
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) {
    phiL[k] = P.phi[k];
    wphiL[k] = P.wphi[k];
  }
  const int gidx_l = wave * CPW + grp;
  double* lamS = wphiL + Q * kp + static_cast<size_t>(gidx_l) * Cfg::group_doubles(Q);  // [NP]
  double* US = lamS + NP;         // [Q][M]
  double* JS = US + Q * M;        // [Q][NJ]
  double* cA = JS + Q * NJ;       // [2][NP] pivot column
  double* cX = cA + 2 * NP;       // [2] pivot row's right-hand side
  double* cP = cX + 2;            // [NP] pivots
  double* stats = wphiL + Q * kp + static_cast<size_t>(waves) * CPW * Cfg::group_doubles(Q);
  __syncthreads();

  int its = 0;
  unsigned status = 0;
  double sx = 0.0, sy = 0.0;
  if (cell >= 0) {
    const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
    const int nc = Nc * M;
    const int i = r / M, a = r % M;
    const bool live = r < nc;
    const size_t gidx = static_cast<size_t>(cell) * M * N + static_cast<size_t>(a) * N + i;
    double lam_r = live ? P.lam[gidx] : 0.0;
    const double uh_r = live ? P.uhat[gidx] : 0.0;

    lamS[r] = lam_r;
    wave_sync();
    double ssum = 0.0;
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (grp * G));
    auto group_all = [&](int v) -> int { return (__ballot(!v) & gmask) == 0ull ? 1 : 0; };
    int ok = group_all(eval_nodes<M>(P, lamS, Nc, phiL, wphiL, r, G, US, JS, ssum));
    wave_sync();

    auto gradient = [&](double& g_out) -> double {
      double g = 0.0;
      if (live)
        for (int q = 0; q < Q; ++q) g = fma(US[q * M + a], wphiL[q * kp + i], g);
      g = live ? g - uh_r : 0.0;
      g_out = g;
      // sum over variables of the Euclidean norm over modes (eq:tauCrit)
      double res = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) res += sqrt(group_sum<G>((a == b) ? g * g : 0.0));
      return res;
    };

    double g_r = 0.0;
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
      // ---- Hessian row in registers; identity beyond the nc unknowns
      double row[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) row[c] = 0.0;
      {
        const double live_f = live ? 1.0 : 0.0;
        int aidx[M];
#pragma unroll
        for (int b = 0; b < M; ++b) aidx[b] = Packed<M>::idx(a, b);
        for (int q = 0; q < Q; ++q) {
          const double wi = wphiL[q * kp + i] * live_f;
          const double* Jq = JS + q * NJ;
          double sb[M];
#pragma unroll
          for (int b = 0; b < M; ++b) sb[b] = Jq[aidx[b]] * wi;
          const double* ph = phiL + q * kp;  // same address in every lane: broadcast
#pragma unroll
          for (int c = 0; c < NP; ++c) row[c] = fma(sb[c % M], ph[c / M], row[c]);
        }
#pragma unroll
        for (int c = 0; c < NP; ++c) row[c] = (live && c < nc) ? row[c] : (c == r ? 1.0 : 0.0);
      }
      // ---- Gauss-Jordan solve H d = g: the pivot row equals the pivot
      // column in the symmetric Schur complement, one LDS broadcast per step
      double x = g_r;
      int pd_ok = 1;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        // steps beyond the cell's unknowns would only touch the identity
        // block; skipping them also bounds the scheduler's window per step
        if (k < nc) {
          double* A = cA + (k & 1) * NP;
          A[r] = row[k];
          if (r == k) cX[k & 1] = x;
          wave_sync();
          const double piv = A[k];
          const double gk = cX[k & 1];
          pd_ok &= piv > 0.0 ? 1 : 0;
          if (r == k) cP[k] = piv;
          const double f = (r == k) ? 0.0 : row[k] * recip(piv);
#pragma unroll
          for (int j = k + 1; j < NP; ++j) row[j] = fma(-f, A[j], row[j]);
          x = fma(-f, gk, x);
        }
      }
      if (!group_all(pd_ok)) {
        status |= kStCholesky;
        break;
      }
      wave_sync();
      const double d_r = live ? x * recip(cP[r]) : 0.0;
      // ---- step length
      const bool ls = !P.one_shot && res > 1e-6;
      double L0 = 0.0, slope = 0.0;
      if (ls) {
        L0 = group_sum<G>(ssum - lam_r * uh_r);
        slope = group_sum<G>(g_r * d_r);
      }
      double t = 1.0, lt_r = lam_r;
      int accepted = 0;
#pragma unroll 1
      for (int h = 0; h <= 60; ++h) {
        lt_r = lam_r - t * d_r;
        lamS[r] = lt_r;
        wave_sync();
        ssum = 0.0;
        ok = group_all(eval_nodes<M>(P, lamS, Nc, phiL, wphiL, r, G, US, JS, ssum));
        wave_sync();
        if (!ls) {
          accepted = 1;
          break;
        }
        if (ok) {
          const double Lt = group_sum<G>(ssum - lt_r * uh_r);
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
    if (live) P.lam[gidx] = lam_r;
    for (int q = r; q < Q; q += G) {
      double u[M];
#pragma unroll
      for (int b = 0; b < M; ++b) u[b] = US[q * M + b];
#pragma unroll
      for (int b = 0; b < M; ++b) P.nodal[(static_cast<size_t>(cell) * Q + q) * M + b] = u[b];
      double ax, ay;
      wave_speeds<M>(P.cp.gamma, P.dim, u, ax, ay);
      sx = nan_max(sx, ax);
      sy = nan_max(sy, ay);
    }
  }

  // ---- per-block statistics: cumulative counters, one slot atomic per direction
  sx = wave_max(sx);
  sy = wave_max(sy);
  if (r == 0) {
    stats[(wave * CPW + grp) * 2 + 0] = static_cast<double>(its);
    stats[(wave * CPW + grp) * 2 + 1] = static_cast<double>(status);
  }
  if (lane == 0) {
    stats[2 * waves * CPW + 2 * wave] = sx;
    stats[2 * waves * CPW + 2 * wave + 1] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum_its = 0, max_its = 0;
    unsigned st = 0;
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < waves * CPW; ++k) {
      const unsigned long long it = static_cast<unsigned long long>(stats[2 * k]);
      sum_its += it;
      max_its = it > max_its ? it : max_its;
      st |= static_cast<unsigned>(stats[2 * k + 1]);
    }
    for (int w = 0; w < waves; ++w) {
      mx = nan_max(mx, stats[2 * waves * CPW + 2 * w]);
      my = nan_max(my, stats[2 * waves * CPW + 2 * w + 1]);
    }
    const int slot = (blockIdx.x & (kSlots - 1)) * kSlotStride;
    if (P.mode == 0) {
      unsigned long long* bs = P.blk_stats + 2 * blockIdx.x;
      bs[0] += sum_its;
      if (max_its > bs[1]) bs[1] = max_its;
      if (st) atomicOr(&P.ctrl->status, st);
      atomicMax(&P.ctrl->amax[P.parity][0][slot], speed_bits(mx));
      if (P.dim == 2) atomicMax(&P.ctrl->amax[P.parity][1][slot], speed_bits(my));
    } else {
      if (st) atomicOr(&P.ctrl->setup_status, st);
      // speeds of the converged initial state feed the first time step
      atomicMax(&P.ctrl->amax[0][0][slot], speed_bits(mx));
      if (P.dim == 2) atomicMax(&P.ctrl->amax[0][1][slot], speed_bits(my));
    }
  }
}

}  // namespace ipm
