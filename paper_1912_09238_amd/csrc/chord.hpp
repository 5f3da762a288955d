// Chord steps of the inexact-Hessian Newton on the register-row layout.
//
// With stored inverse Hessians (the outlook of Sec. 7 on not recomputing the
// Hessian) almost every Newton iteration (eq:dualIteration1) takes its step
// from the cell's stored -H^-1: the ansatz and the gradient of eq:L at the
// nodes, the tau test of eq:tauCrit, one matrix-vector product and the line
// search of the step length.  None of that needs the Hessian row a lane of
// the full kernel (dual.hpp) keeps in registers for assembly and inversion,
// so this kernel runs those iterations alone, with a small register and LDS
// footprint: many more wavefronts per CU.
//
// Per listed cell: while the cell has a valid stored inverse, iterate chord
// steps exactly as the full kernel does (same arithmetic in the same order:
// the nodes stream through in chunks, node by node in ascending order; the
// matrix-vector sum over columns in ascending order).  A cell whose inverse
// is missing, or whose step fails to contract the dual residual by theta,
// is handed on (hinv_ok = 2, appended to the class's list of handed-on
// cells) with its dual written back; the full kernel, launched next in
// pending mode over that list, continues it from there with a fresh
// Hessian.  Layout: a group of G = NP lanes per
// cell, lane r holds unknown r = i M + a.
#pragma once

#include "dual.hpp"

namespace ipm {

// Secant pairs kept per cell within a launch: the step applies the stored
// inverse with the L-BFGS two-loop corrections of the cell's last accepted
// steps (0: plain chord steps).
constexpr int kChordPairs = 1;

template <int M, int NP>
struct ChordCfg {
  static constexpr int G = NP;
  static constexpr int CPW = 64 / G;
  static constexpr int NJ = M * (M + 1) / 2;
  // nodes per chunk: one per lane, as the full kernel (the same lanes sum
  // the same nodes, so both kernels round alike)
  __host__ __device__ static int chunk(int Q) { return Q < G ? Q : G; }
  // one cell per wavefront and at most two chunks: the ansatz of every node
  // stays in LDS after a pass (the write-back of the final dual's nodal
  // ansatz reads it instead of evaluating the closure again)
  __host__ __device__ static bool keep_all(int Q) { return CPW == 1 && Q <= 2 * G; }
  // per group: dual [NP], ansatz [CH][M] (keep_all: [Q][M])
  __host__ __device__ static int group_doubles(int Q) {
    return NP + (keep_all(Q) ? Q : chunk(Q)) * M;
  }
  // node stride of the tables, which are stored mode by mode (a node per
  // lane reads consecutive words); odd, so that lanes of different modes
  // read different banks
  __host__ __device__ static int qstride(int Q) { return Q | 1; }
  // tables Phi and w Phi [kl][Q|1] and w [Q], the groups' areas, 2 stats per
  // group and 2 speeds per wavefront
  __host__ __device__ static size_t lds_bytes(int Q, int kl, int waves) {
    return sizeof(double) * (2 * static_cast<size_t>(kl) * qstride(Q) + Q +
                             static_cast<size_t>(waves) * CPW * group_doubles(Q) +
                             2 * static_cast<size_t>(waves) * (CPW + 1));
  }
};

// Sum over the lanes of each residue class mod 4 within aligned groups of G
// = 16, 32 or 64 lanes (rotations by 4 and 8 inside each 16-lane row, then
// exchanges across rows): every lane receives its class's total.
template <int G>
__device__ __forceinline__ double class4_sum(double v) {
  v += dpp_mov<0x124>(v);  // row_ror:4
  v += dpp_mov<0x128>(v);  // row_ror:8
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// The residual of the tau test, sum over the m = 4 variables of the
// Euclidean norm of the gradient over the modes, for a group whose lane r
// holds unknown (i, a) with a = r mod 4: one class sum and one square root
// per lane, the four norms then added within each quad (the same value in
// every lane: addition commutes).
template <int G>
__device__ __forceinline__ double tau_residual4_sq(double g2) {
  const double s = sqrt(class4_sum<G>(g2));
  const double t = s + dpp_mov<0xB1>(s);
  return t + dpp_mov<0x4E>(t);
}
template <int G>
__device__ __forceinline__ double tau_residual4(double g) {
  return tau_residual4_sq<G>(g * g);
}

// A cell's counters in one double (exact below 2^53): iterations (10 bits),
// passes over the nodes (30 bits), listed flag.
__device__ __forceinline__ double pack_stats(int its, int evals, bool listed) {
  return static_cast<double>(static_cast<unsigned long long>(its) |
                             (static_cast<unsigned long long>(evals) << 10) |
                             (listed ? (1ull << 40) : 0ull));
}

// Hand a cell on to the full kernel: marked (hinv_ok = 2, no valid inverse)
// and appended to its class's list for this step.
__device__ __forceinline__ void hand_on(const DualParams& P, int cell) {
  P.hinv_ok[cell] = 2;
  const unsigned k = atomicAdd(&P.ctrl->pend_len[P.parity][P.cls], 1u);
  P.pend_list[k] = cell;
}

// Ansatz value u_s(lambda^T phi(xi_q)) of one node (no Jacobian); phi_i(q)
// at ph[i * stride].
template <int M>
__device__ __forceinline__ bool node_ansatz(const DualParams& P, const double* lamS, int Nc,
                                            const double* ph, int stride, double (&u)[M],
                                            double& ss) {
  constexpr int NJ = M * (M + 1) / 2;
  double L[M], J[NJ];
#pragma unroll
  for (int a = 0; a < M; ++a) L[a] = 0.0;
#pragma unroll 4
  for (int i = 0; i < Nc; ++i) {
    const double f = ph[i * stride];
#pragma unroll
    for (int a = 0; a < M; ++a) L[a] = fma(lamS[i * M + a], f, L[a]);
  }
  return closure<M>(P.cp, L, u, J, ss);
}

template <int M, int NP>
__device__ __forceinline__ void chord_body(const DualParams& P, const int blk) {
  using Cfg = ChordCfg<M, NP>;
  constexpr int G = Cfg::G, CPW = Cfg::CPW;
  const bool stop = P.mode == 0 && ((P.ctrl->done[P.parity] != 0) | (P.ctrl->status != 0u));
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G;
  const int r = lane % G;
  int cell = work_cell(P, (blk * waves + wave) * CPW + grp);
  if (stop) return;  // uniform
  if (P.mode == 0 && P.reset_next && blk == 0) reset_next_step(P);
  // a cell without a valid stored inverse goes to the full kernel at once
  if (cell >= 0 && P.hinv_ok[cell] != 1) {
    if (r == 0) hand_on(P, cell);
    cell = -1;
  }
  if (!__syncthreads_or(cell >= 0)) return;

  const int Q = P.Q, kg = P.kp, kp = P.kl, N = P.N;
  // one cell per wavefront: its size is wave-uniform (scalar loop control)
  int Nc = cell >= 0 ? (P.cellN ? static_cast<int>(P.cellN[cell]) : N) : 0;
  if (CPW == 1) Nc = __builtin_amdgcn_readfirstlane(Nc);
  const int nc = Nc * M;
  const int ii = r / M, aa = r % M;
  const bool live = r < nc;
  const size_t gidx = static_cast<size_t>(cell >= 0 ? cell : 0) * M * N + static_cast<size_t>(aa) * N + ii;
  double lam = live ? P.lam[gidx] : 0.0;
  const double uh = live ? P.uhat[gidx] : 0.0;
  extern __shared__ double smem[];
  const int QT = Cfg::qstride(Q);
  double* phiT = smem;             // [kp][QT]: phi_i(q)
  double* wphiT = phiT + kp * QT;  // [kp][QT]: w_q phi_i(q)
  double* wL = wphiT + kp * QT;    // [Q]
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) {
    const int q = k / kp, i = k % kp;
    phiT[i * QT + q] = P.phi[q * kg + i];
    wphiT[i * QT + q] = P.wphi[q * kg + i];
  }
  for (int q = threadIdx.x; q < Q; q += blockDim.x) wL[q] = P.wphi[static_cast<size_t>(q) * kg];
  const int CH = Cfg::chunk(Q);
  double* areas = wL + Q;
  double* lamS = areas + static_cast<size_t>(wave * CPW + grp) * Cfg::group_doubles(Q);  // [NP]
  double* US = lamS + NP;  // [CH][M], keep_all: [Q][M]
  const bool keep = Cfg::keep_all(Q);
  double* stats = areas + static_cast<size_t>(waves) * CPW * Cfg::group_doubles(Q);
  __syncthreads();

  int its = 0, evals = 0;  // evals: passes over the nodes (entry and each trial)
  unsigned status = 0;
  bool pending = false;
  double sx = 0.0, sy = 0.0;
  if (cell >= 0) {
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (grp * G));
    auto group_all = [&](int v) -> int { return (__ballot(!v) & gmask) == 0ull ? 1 : 0; };
    const global_fptr Hc =
        (global_fptr)(P.hinv + static_cast<size_t>(P.hinv_slot ? P.hinv_slot[cell] : cell) * P.hinv_stride);
    lamS[r] = lam;
    wave_sync();
    // the nodes in chunks (lane r: node c0 + r): <s_*> and the gradient sum
    // of this lane's unknown, node by node in ascending order
    double ssum = 0.0, gacc = 0.0;
    auto grad_pass = [&]() -> int {
      ++evals;
      int okp = 1;
      ssum = 0.0;
      gacc = 0.0;
      for (int c0 = 0; c0 < Q; c0 += CH) {
        const int q = c0 + r;
        if (q < Q) {
          double u[M], ss;
          okp &= node_ansatz<M>(P, lamS, Nc, phiT + q, QT, u, ss) ? 1 : 0;
#pragma unroll
          for (int a = 0; a < M; ++a) US[(keep ? q : r) * M + a] = u[a];
          ssum = fma(wL[q], ss, ssum);
        }
        wave_sync();
        const int nq = Q - c0 < CH ? Q - c0 : CH;
        // w_q phi_i(q) is the product the host formed once (phi_0 = 1, so
        // wL holds w_q exactly and the terms equal wL[q] * phi_i(q))
        if (live) {
          const double* wr = wphiT + ii * QT + c0;
          const double* uc = keep ? US + c0 * M : US;
          for (int j = 0; j < nq; ++j) gacc = fma(uc[j * M + aa], wr[j], gacc);
        }
        wave_sync();
      }
      return okp;
    };
    double g = 0.0;
    auto norm = [&]() -> double {
      if constexpr (M == 4 && G >= 16) return tau_residual4<G>(g);
      double res = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) res += sqrt(group_sum<G>(aa == b ? g * g : 0.0));
      return res;
    };
    auto gradient = [&]() -> double {
      g = live ? gacc - uh : 0.0;
      return norm();
    };
    // the previous update's warm start (Euler entropy): the gradient and
    // <s_*> at this dual, which spares the entry pass over the nodes
    const bool warm = P.gwarm != nullptr && P.ctrl->gwarm[P.parity] != 0;  // uniform
    bool entry_warm = warm;
    double s0 = 0.0;
    int ok = 1;
    double res = 0.0;
    if (warm) {
      g = live ? P.gwarm[gidx] : 0.0;
      res = norm();
      s0 = P.s0[cell];
    } else {
      ok = group_all(grad_pass());
      if (ok) res = gradient();
      else status |= kStRealizability;
    }
    // secant pairs s = lambda_k+1 - lambda_k, y = g_k+1 - g_k of this launch,
    // oldest first in the last npair slots, with rho = 1 / (y . s)
    constexpr int KP = kChordPairs > 0 ? kChordPairs : 1;
    double sp[KP], yp[KP], rho[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) sp[k] = yp[k] = rho[k] = 0.0;
    int npair = 0;
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
      // ---- d = H^-1 g = -(rows of -H^-1) g, g through the group's LDS area;
      // with secant pairs, the two-loop recursion around the stored inverse
      double qv = g, alpha[KP];
      if (kChordPairs > 0) {
#pragma unroll
        for (int k = KP - 1; k >= 0; --k) {
          alpha[k] = 0.0;
          if (k >= KP - npair) {  // uniform
            alpha[k] = rho[k] * group_sum<G>(sp[k] * qv);
            qv = fma(-alpha[k], yp[k], qv);
          }
        }
      }
      lamS[r] = qv;
      wave_sync();
      // the stored entries of B columns requested at once, then summed in
      // ascending column order.  Loads are unconditional: a column past nc
      // re-reads the last one, and its product with the zero that lamS holds
      // there (g = 0 beyond nc, B divides NP) adds nothing.
      constexpr int B = NP < 16 ? NP : 16;
      double acc = 0.0;
      if (live) {
        const global_fptr hp = Hc + r;
        for (int c0 = 0; c0 < nc; c0 += B) {
          float h[B];
#pragma unroll
          for (int j = 0; j < B; ++j) h[j] = hp[min(c0 + j, nc - 1) * nc];
#pragma unroll
          for (int j = 0; j < B; ++j) acc = fma(static_cast<double>(h[j]), lamS[c0 + j], acc);
        }
      }
      double d = live ? -acc : 0.0;
      if (kChordPairs > 0) {
#pragma unroll
        for (int k = 0; k < KP; ++k)
          if (k >= KP - npair) {  // uniform
            const double beta = rho[k] * group_sum<G>(yp[k] * d);
            d = fma(sp[k], alpha[k] - beta, d);
          }
      }
      wave_sync();
      // ---- step length (as the full kernel: backtracking while far from tau)
      const bool ls = !P.one_shot && res > 1e-6;
      double L0 = 0.0, slope = 0.0;
      if (ls) {
        L0 = entry_warm ? s0 - group_sum<G>(lam * uh) : group_sum<G>(ssum - lam * uh);
        slope = group_sum<G>(g * d);
      }
      entry_warm = false;  // from here on ssum is the accepted trial's
      double t = 1.0, lt = lam;
      int accepted = 0;
#pragma unroll 1
      for (int h = 0; h <= 60; ++h) {
        lt = lam - t * d;
        lamS[r] = lt;
        wave_sync();
        ok = group_all(grad_pass());
        if (!ls) {
          accepted = 1;
          break;
        }
        if (ok) {
          const double Lt = group_sum<G>(ssum - lt * uh);
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
      const double lam_old = lam, g_old = g;
      lam = lt;
      ++its;
      if (!ok) {
        status |= kStRealizability;
        break;
      }
      const double res_old = res;
      res = gradient();
      if (kChordPairs > 0) {
        const double s_new = lam - lam_old, y_new = g - g_old;
        const double ys = group_sum<G>(s_new * y_new);
        if (ys > 0.0) {  // strictly convex L: always, up to rounding
#pragma unroll
          for (int k = 0; k + 1 < KP; ++k) {
            sp[k] = sp[k + 1];
            yp[k] = yp[k + 1];
            rho[k] = rho[k + 1];
          }
          sp[KP - 1] = s_new;
          yp[KP - 1] = y_new;
          rho[KP - 1] = 1.0 / ys;
          npair = npair < KP ? npair + 1 : KP;
        }
      }
      // no contraction by theta: the inverse is retired; the cell goes on in
      // the full kernel (its next iteration assembles afresh), or, one-shot,
      // at its next pseudo-time step
      if (!(res <= P.reuse_theta * res_old)) {
        if (P.one_shot) {
          if (r == 0) P.hinv_ok[cell] = 0;
        } else {
          pending = true;
        }
        break;
      }
      if (P.one_shot) break;
    }
    // ---- write back: the dual; unless pending, the nodal ansatz of the
    // final dual (once more, node by node) and the wave speeds
    if (live) P.lam[gidx] = lam;
    if (pending || status) {
      if (r == 0 && pending) hand_on(P, cell);
    } else {
      // keep_all and a pass made: the last pass was at the final dual (the
      // accepted trial, or the entry pass of a cell already within tau), and
      // its nodal ansatz is in LDS, the same values bit for bit
      const bool stored = keep && evals > 0;
      for (int q = r; q < Q; q += G) {
        double u[M], ss;
        if (stored) {
#pragma unroll
          for (int b = 0; b < M; ++b) u[b] = US[q * M + b];
        } else {
          (void)node_ansatz<M>(P, lamS, Nc, phiT + q, QT, u, ss);
        }
#pragma unroll
        for (int b = 0; b < M; ++b) P.nodal[(static_cast<size_t>(cell) * Q + q) * M + b] = u[b];
        double ax, ay;
        wave_speeds<M>(P.cp.gamma, P.dim, u, ax, ay);
        sx = nan_max(sx, ax);
        sy = nan_max(sy, ay);
      }
    }
  }

  // ---- per-block statistics and speed slots (as the full kernel)
  sx = wave_max(sx);
  sy = wave_max(sy);
  if (r == 0) {
    stats[(wave * CPW + grp) * 2 + 0] = pack_stats(its, evals, cell >= 0);
    stats[(wave * CPW + grp) * 2 + 1] = static_cast<double>(status);
  }
  if (lane == 0) {
    stats[2 * waves * CPW + 2 * wave] = sx;
    stats[2 * waves * CPW + 2 * wave + 1] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum_its = 0, max_its = 0, listed = 0, sum_evals = 0;
    unsigned st = 0;
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < waves * CPW; ++k) {
      const unsigned long long v = static_cast<unsigned long long>(stats[2 * k]);
      const unsigned long long it = v & 1023ull;
      sum_its += it;
      max_its = it > max_its ? it : max_its;
      sum_evals += (v >> 10) & 0x3fffffffull;
      listed += v >> 40;
      st |= static_cast<unsigned>(stats[2 * k + 1]);
    }
    for (int w = 0; w < waves; ++w) {
      mx = nan_max(mx, stats[2 * waves * CPW + 2 * w]);
      my = nan_max(my, stats[2 * waves * CPW + 2 * w + 1]);
    }
    const int slot = (blk & (kSlots - 1)) * kSlotStride;
    unsigned long long* bs = P.blk_stats + kBlkStats * static_cast<size_t>(blk);
    bs[0] += sum_its;
    if (max_its > bs[1]) bs[1] = max_its;
    bs[2] += listed;
    bs[3] += sum_evals;
    if (st) atomicOr(&P.ctrl->status, st);
    atomicMax(&P.ctrl->amax[P.parity][0][slot], speed_bits(mx));
    if (P.dim == 2) atomicMax(&P.ctrl->amax[P.parity][1][slot], speed_bits(my));
  }
}

// four wavefronts per SIMD (128 registers)
template <int M, int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void newton_chord_kernel(DualParams P) {
  chord_body<M, NP>(P, blockIdx.x);
}

template <int M, int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void newton_chord_batched(const DualParams* __restrict__ PP, const int* __restrict__ begin, int n) {
  const int k = batch_problem(begin, n, blockIdx.x);
  chord_body<M, NP>(PP[k], blockIdx.x - begin[k]);
}

}  // namespace ipm
