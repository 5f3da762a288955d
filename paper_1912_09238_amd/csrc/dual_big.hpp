// Dual Newton solve for cells with more than 64 unknowns (n = m N up to 16 T):
// one 256-thread workgroup per cell.
//
// The steps are those of the small-cell kernel (ansatz eq:ansatz, gradient of
// eq:L and the test eq:tauCrit, Hessian eq:dualIterationFunction, step
// eq:dualIteration1 with the backtracking rule of the line search); only the
// layout differs:
//   - threads over quadrature nodes for the ansatz, over unknowns for the
//     gradient (unknown r = i M + a, as everywhere in this library);
//   - the Hessian as a 16 x 16 grid of T x T register tiles: thread (tr, tc)
//     holds rows tr + 16 i and columns tc + 16 j.  Since M divides 16, all
//     rows of a tile share the variable a = tr mod M and all columns the
//     variable b = tc mod M, so a tile's entries take one entry J_ab of the
//     closure Jacobian per node and the sum over nodes is a rank-1 update;
//   - precision form (PREC = 1): each unique block H_ab = Phi^T diag(w J_ab)
//     Phi (symmetric in the mode indices, H_ab = H_ba) is a matrix product
//     on the MFMA units, v_mfma_f32_16x16x32_bf16 with FP32 accumulation;
//     both operands are split into BF16 high and low parts and three
//     products are summed (about 16 significant bits).  The blocks land in
//     LDS and every thread gathers its FP64 tile.  Gradient, tau test and the
//     solve stay FP64, so the Newton loop still stops at the FP64 tolerance;
//   - Gauss-Jordan without pivoting (H is SPD): the owners of the pivot
//     column publish it to LDS, one barrier per step; every thread reads the
//     column entries of its rows (multipliers) and, by symmetry of the
//     trailing Schur complement, of its columns (the pivot row).  Only
//     columns right of the pivot are updated: the eliminated pivot rows above
//     are no longer symmetric with their columns;
//   - inexact-Hessian Newton (hinv set; the outlook of Sec. 7 on not
//     recomputing the Hessian): a fresh assembly is inverted in place by
//     Gauss-Jordan (both the pivot row and the pivot column are published,
//     as the partly inverted matrix is not symmetric), the inverse's tiles
//     are kept in HBM, and later Newton iterations of the cell, in this and
//     in following steps, take d = H_old^-1 g from them while each such
//     iteration contracts the dual residual by a factor theta; otherwise the inverse is
//     retired and the next iteration (one-shot: of the next pseudo-time
//     step) assembles and inverts afresh.  The tau test stays exact, so
//     the iteration stops at the same FP64 tolerance.
#pragma once

#include "dual.hpp"

namespace ipm {

template <int M, int T, int PREC = 0>
struct BigCfg {
  static_assert(16 % M == 0, "tile variables need M | 16");
  static constexpr int NPB = 16 * T;  // unknowns incl. identity padding
  // 16-mode tiles of one variable's block: the class's cells have at most
  // 16 T / M modes, whatever the problem's widest cell
  static constexpr int NTMAX = (16 * T / M + 15) / 16;
  __host__ __device__ static int block_tiles(int kp) {
    const int nt = (kp + 15) / 16;
    return nt < NTMAX ? nt : NTMAX;
  }
  static constexpr int NJ = M * (M + 1) / 2;
  // inexact-Hessian Newton: right-hand side [NPB] and row partial sums
  // [16][NPB] of the product with the stored inverse, after the rest
  __host__ __device__ static size_t reuse_bytes() { return sizeof(double) * 17 * NPB; }
  __host__ __device__ static size_t lds_bytes(int Q, int kp, bool bcache = true) {
    // phi [Q][kp]; w [Q]; lam [NPB]; U [Q][M]; J [Q][NJ]; column [2][NPB];
    // pivot-row rhs [2]; reduction scratch [4][8]
    size_t b = sizeof(double) * (static_cast<size_t>(Q) * kp + Q + NPB +
                                 static_cast<size_t>(Q) * (M + NJ) + 2 * NPB + 2 + 32);
    if (PREC & 1) {
      // FP32 blocks [NJ][16 NT][16 NT] and BF16 hi/lo B fragments
      // [NT][QC][64 lanes][16], NT = ceil(N / 16) for the class's widest
      // cell, QC = ceil(Q / 32)
      const size_t nt = block_tiles(kp), qc = (Q + 31) / 32;
      b += sizeof(float) * NJ * (16 * nt) * (16 * nt) + (bcache ? 32 * 64 * nt * qc : 0);
    }
    return b;
  }
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x = hi + lo with hi, lo in BF16 (round to nearest): hi carries 8
// significant bits, hi + lo about 16
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

// Sum over the workgroup (256 threads, all active) of K values per thread.
// Fixed reduction order: identical results in every thread and every run.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[w * 8 + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = (red[k] + red[8 + k]) + (red[16 + k] + red[24 + k]);
  __syncthreads();
}

template <int M, int T, int PREC>
__device__ __forceinline__ void newton_big_body(const DualParams& P, const int blk) {
  using Cfg = BigCfg<M, T, PREC>;
  constexpr int NPB = Cfg::NPB, NJ = Cfg::NJ;
  // the stop flags are read with the list lengths (one round trip, not two)
  const bool stop = P.mode == 0 && ((P.ctrl->done[P.parity] != 0) | (P.ctrl->status != 0u));
  int cell = work_cell(P, blk);
  if (stop) return;  // uniform
  if (P.mode == 0 && P.reset_next && blk == 0) reset_next_step(P);
  if (cell < 0) return;  // uniform over the workgroup

  // kp: LDS stride of the staged table (the class's columns), kg: the
  // global table's
  const int Q = P.Q, kg = P.kp, kp = P.kl, N = P.N;
  const int tid = threadIdx.x;
  extern __shared__ double smem[];
  double* phiL = smem;
  double* wL = phiL + Q * kp;      // [Q] weights (w phi_0, phi_0 = 1)
  double* lamS = wL + Q;           // [NPB]
  double* US = lamS + NPB;         // [Q][M]
  double* JS = US + Q * M;         // [Q][NJ]
  double* col = JS + Q * NJ;       // [2][NPB]
  double* xk = col + 2 * NPB;      // [2]
  double* red = xk + 2;            // [32]
  for (int k = tid; k < Q * kp; k += 256) phiL[k] = P.phi[(k / kp) * kg + k % kp];
  for (int q = tid; q < Q; q += 256) wL[q] = P.wphi[static_cast<size_t>(q) * kg];
  // precision form: FP32 Hessian blocks and the constant B fragments phi_k(q)
  const int NT = Cfg::block_tiles(kp), QC = (Q + 31) / 32, S16 = 16 * NT;
  float* Hb = reinterpret_cast<float*>(red + 32);                        // [NJ][S16][S16]
  bf16x8* Bf = reinterpret_cast<bf16x8*>(Hb + static_cast<size_t>(NJ) * S16 * S16);  // [NT][QC][2][64]
  // B fragment f = K QC + c of this lane: phi_k(q) for its column k and 8 nodes
  auto b_fragment = [&](int f, bf16x8& hi, bf16x8& lo) {
    const int K = f / QC, c = f % QC, lane = tid & 63;
    const int k = K * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = c * 32 + 8 * (lane >> 4) + j;
      const float v = (q < Q && k < N && k < kp) ? static_cast<float>(phiL[q * kp + k]) : 0.0f;
      __bf16 h, l;
      split_bf16(v, h, l);
      hi[j] = h;
      lo[j] = l;
    }
  };
  if constexpr ((PREC & 1) != 0) {
    __syncthreads();  // phiL is complete
    if (P.bcache)
      for (int f = tid >> 6; f < NT * QC; f += 4) {
        const int lane = tid & 63;
        bf16x8 hi, lo;
        b_fragment(f, hi, lo);
        Bf[(static_cast<size_t>(f) * 2) * 64 + lane] = hi;
        Bf[(static_cast<size_t>(f) * 2 + 1) * 64 + lane] = lo;
      }
  }

  const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
  const int nc = Nc * M;
  // unknown owned by this thread (gradient, right-hand side, step)
  const bool row_live = tid < nc;
  const int ri = tid / M, ra = tid % M;
  const size_t gidx = static_cast<size_t>(cell) * M * N + static_cast<size_t>(ra) * N + ri;
  double lam = row_live ? P.lam[gidx] : 0.0;
  const double uh = row_live ? P.uhat[gidx] : 0.0;
  if (tid < NPB) lamS[tid] = row_live ? lam : 0.0;
  __syncthreads();

  // tile coordinates
  const int tr = tid >> 4, tc = tid & 15;
  const int jidx = Packed<M>::idx(tr % M, tc % M);

  int its = 0, nfresh = 0;
  unsigned status = 0;
  double ssum = 0.0;
  int ok = eval_nodes<M>(P, lamS, Nc, phiL, wL, 1, tid, 256, US, JS, ssum);
  ok = __syncthreads_and(ok);

  double g = 0.0;
  auto gradient = [&]() -> double {
    double gg = 0.0;
    if (row_live) {
      for (int q = 0; q < Q; ++q) gg = fma(US[q * M + ra] * wL[q], phiL[q * kp + ri], gg);
      gg -= uh;
    }
    g = gg;
    double e2[M];
#pragma unroll
    for (int b = 0; b < M; ++b) e2[b] = (row_live && ra == b) ? gg * gg : 0.0;
    block_sum<M>(e2, red);
    double res = 0.0;
#pragma unroll
    for (int b = 0; b < M; ++b) res += sqrt(e2[b]);
    return res;
  };

  double res = 0.0;
  if (ok) res = gradient();
  else status |= kStRealizability;

  // inexact-Hessian Newton: LDS after the kernel's other areas, or, with the
  // MFMA Hessian, the FP32 block area, which is free once the tiles are
  // gathered
  double* mvL = ((PREC & 1) != 0)
                    ? reinterpret_cast<double*>(Hb)
                    : reinterpret_cast<double*>(reinterpret_cast<char*>(smem) +
                                                Cfg::lds_bytes(Q, kp, P.bcache != 0));
  double* gS = mvL;                // [NPB] right-hand side
  double* part = mvL + NPB;        // [16][NPB] row partial sums
  double* rowb = part;             // [2][NPB] pivot rows during the inversion
  bool chord = true;
  // the cell's stored inverse is valid: read once, then kept in step with
  // the flag this cell writes (no re-read of its own write)
  bool have_inv = false;
  if constexpr ((PREC & 2) != 0) have_inv = P.hinv_ok[cell] == 1;
  // d (unknown tid) = sum_c Hinv[tid][c] g[c] from the register tiles, the
  // column sums taken in a fixed order
  auto inverse_times = [&](const double (&A)[T][T], double gv) -> double {
    if (tid < NPB) gS[tid] = row_live ? gv : 0.0;
    __syncthreads();
    double gc[T];
#pragma unroll
    for (int j = 0; j < T; ++j) gc[j] = gS[tc + 16 * j];
#pragma unroll
    for (int i = 0; i < T; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < T; ++j) s = fma(A[i][j], gc[j], s);
      part[tc * NPB + tr + 16 * i] = s;
    }
    __syncthreads();
    double dv = 0.0;
    if (tid < NPB)
      for (int c = 0; c < 16; ++c) dv += part[c * NPB + tid];
    __syncthreads();
    return row_live ? dv : 0.0;
  };

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
    // ---- inexact-Hessian Newton: the stored inverse while it contracts
    constexpr bool reuse = (PREC & 2) != 0;  // inexact-Hessian variant
    const bool stale = reuse && chord && have_inv;  // uniform
    double d = 0.0;
    double H[T][T];
    float* Hc = reuse ? P.hinv + static_cast<size_t>(P.hinv_slot ? P.hinv_slot[cell] : cell) *
                                      P.hinv_stride
                       : nullptr;
    if (stale) {
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) H[i][j] = static_cast<double>(Hc[(i * T + j) * 256 + tid]);
      d = inverse_times(H, g);
    } else {
    // ---- Hessian tiles
    if constexpr ((PREC & 1) != 0) {
      // blocks H_ab[i][k] = sum_q w_q J_ab(q) phi_i(q) phi_k(q) on the MFMA
      // units: task (ab, I) builds the A fragments of row tile I once per
      // chunk of 32 nodes and runs all column tiles K
      const int lane = tid & 63, NTc = (Nc + 15) / 16;
      for (int task = tid >> 6; task < NJ * NTc; task += 4) {
        const int ab = task / NTc, I = task % NTc;
        const int i = I * 16 + (lane & 15);
        constexpr int KT = (T + M - 1) / M;  // column tiles of the largest N of the class
        f32x4 acc[KT];
#pragma unroll
        for (int K = 0; K < KT; ++K) acc[K] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < QC; ++c) {
          bf16x8 ahi, alo;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const int q = c * 32 + 8 * (lane >> 4) + j;
            const float v = (q < Q && i < Nc)
                                ? static_cast<float>(wL[q] * JS[q * NJ + ab] * phiL[q * kp + i])
                                : 0.0f;
            __bf16 h, l;
            split_bf16(v, h, l);
            ahi[j] = h;
            alo[j] = l;
          }
#pragma unroll
          for (int K = 0; K < KT; ++K) {
            if (K < NTc) {
              const size_t f = static_cast<size_t>(K) * QC + c;
              bf16x8 bhi, blo;
              if (P.bcache) {
                bhi = Bf[(f * 2) * 64 + lane];
                blo = Bf[(f * 2 + 1) * 64 + lane];
              } else {
                b_fragment(static_cast<int>(f), bhi, blo);
              }
              acc[K] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc[K], 0, 0, 0);
              acc[K] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc[K], 0, 0, 0);
              acc[K] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc[K], 0, 0, 0);
            }
          }
        }
#pragma unroll
        for (int K = 0; K < KT; ++K)
          if (K < NTc)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              Hb[(static_cast<size_t>(ab) * S16 + I * 16 + 4 * (lane >> 4) + r) * S16 + K * 16 +
                 (lane & 15)] = acc[K][r];
      }
      __syncthreads();
      const int ab = Packed<M>::idx(tr % M, tc % M);
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const int r = tr + 16 * i, c = tc + 16 * j;
          H[i][j] = (r < nc && c < nc)
                        ? static_cast<double>(Hb[(static_cast<size_t>(ab) * S16 + r / M) * S16 + c / M])
                        : (r == c ? 1.0 : 0.0);
        }
      if constexpr (reuse) __syncthreads();  // the inversion reuses the block area
    } else {
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) H[i][j] = 0.0;
      {
        int li[T], lj[T];
        double mi[T], mj[T];
#pragma unroll
        for (int i = 0; i < T; ++i) {
          const int r = tr + 16 * i;
          li[i] = r < nc ? r / M : 0;
          mi[i] = r < nc ? 1.0 : 0.0;
        }
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const int c = tc + 16 * j;
          lj[j] = c < nc ? c / M : 0;
          mj[j] = c < nc ? 1.0 : 0.0;
        }
        for (int q = 0; q < Q; ++q) {
          const double s = JS[q * NJ + jidx] * wL[q];
          double lv[T], rv[T];
#pragma unroll
          for (int i = 0; i < T; ++i) lv[i] = phiL[q * kp + li[i]] * (s * mi[i]);
#pragma unroll
          for (int j = 0; j < T; ++j) rv[j] = phiL[q * kp + lj[j]] * mj[j];
#pragma unroll
          for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j) H[i][j] = fma(lv[i], rv[j], H[i][j]);
        }
        // identity beyond the cell's unknowns
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
          for (int j = 0; j < T; ++j) {
            const int r = tr + 16 * i, c = tc + 16 * j;
            if (r >= nc || c >= nc) H[i][j] = (r == c) ? 1.0 : 0.0;
          }
      }
    }
    if constexpr (reuse) {
      // ---- in-place Gauss-Jordan inversion H <- H^-1 (SPD, no pivoting)
      int pd_ok = 1;
#pragma unroll
      for (int jb = 0; jb < T; ++jb) {
        for (int kk = 0; kk < 16; ++kk) {
          const int k = jb * 16 + kk;
          if (k >= nc) break;  // uniform
          double* cb = col + (k & 1) * NPB;          // pivot column
          double* rw = rowb + (k & 1) * NPB;         // pivot row
          if (tc == kk) {
#pragma unroll
            for (int i = 0; i < T; ++i) cb[tr + 16 * i] = H[i][jb];
          }
          if (tr == kk) {
#pragma unroll
            for (int j = 0; j < T; ++j) rw[tc + 16 * j] = H[jb][j];
          }
          __syncthreads();
          const double piv = cb[k];
          pd_ok &= piv > 0.0 ? 1 : 0;
          const double rp = recip(piv);
          double cr[T], rc[T];
#pragma unroll
          for (int i = 0; i < T; ++i) cr[i] = cb[tr + 16 * i] * rp;
#pragma unroll
          for (int j = 0; j < T; ++j) rc[j] = rw[tc + 16 * j];
#pragma unroll
          for (int i = 0; i < T; ++i)
#pragma unroll
            for (int j = 0; j < T; ++j) {
              const int r = tr + 16 * i, c = tc + 16 * j;
              const double upd = fma(-cr[i], rc[j], H[i][j]);
              H[i][j] = (r == k) ? ((c == k) ? rp : rc[j] * rp) : ((c == k) ? -cr[i] : upd);
            }
        }
      }
      if (!pd_ok) {  // uniform: every thread read the same pivots
        status |= kStPivot;
        break;
      }
#pragma unroll
      for (int i = 0; i < T; ++i)
#pragma unroll
        for (int j = 0; j < T; ++j) Hc[(i * T + j) * 256 + tid] = static_cast<float>(H[i][j]);
      if (tid == 0) P.hinv_ok[cell] = 1;
      have_inv = true;
      d = inverse_times(H, g);
    } else {
    // ---- Gauss-Jordan solve H d = g
    double x = g, dg = 1.0;
    int pd_ok = 1;
#pragma unroll
    for (int jb = 0; jb < T; ++jb) {
      for (int kk = 0; kk < 16; ++kk) {
        const int k = jb * 16 + kk;
        if (k >= nc) break;  // uniform
        double* cb = col + (k & 1) * NPB;
        if (tc == kk) {
#pragma unroll
          for (int i = 0; i < T; ++i) cb[tr + 16 * i] = H[i][jb];
        }
        if (tid == k) xk[k & 1] = x;
        __syncthreads();
        const double piv = cb[k];
        const double gk = xk[k & 1];
        pd_ok &= piv > 0.0 ? 1 : 0;
        const double rp = recip(piv);
        double f[T], pr[T];
#pragma unroll
        for (int i = 0; i < T; ++i) {
          const int r = tr + 16 * i;
          f[i] = (r == k) ? 0.0 : cb[r] * rp;
        }
        // column blocks before the pivot's are eliminated already
#pragma unroll
        for (int j = jb; j < T; ++j) {
          const int c = tc + 16 * j;
          pr[j] = (c > k) ? cb[c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < T; ++i)
#pragma unroll
          for (int j = jb; j < T; ++j) H[i][j] = fma(-f[i], pr[j], H[i][j]);
        if (tid < NPB) {
          if (tid == k) dg = piv;
          else x = fma(-(cb[tid] * rp), gk, x);
        }
      }
    }
    if (!pd_ok) {  // uniform: every thread read the same pivots
      status |= kStPivot;
      break;
    }
    d = row_live ? x * recip(dg) : 0.0;
    }  // exact solve
    }  // fresh Hessian
    // ---- step length
    const bool ls = !P.one_shot && res > 1e-6;
    double L0 = 0.0, slope = 0.0;
    if (ls) {
      double v2[2] = {ssum - (row_live ? lam * uh : 0.0), row_live ? g * d : 0.0};
      block_sum<2>(v2, red);
      L0 = v2[0];
      slope = v2[1];
    }
    double t = 1.0, lt = lam;
    int accepted = 0;
#pragma unroll 1
    for (int h = 0; h <= 60; ++h) {
      lt = lam - t * d;
      if (tid < NPB) lamS[tid] = row_live ? lt : 0.0;
      __syncthreads();
      ssum = 0.0;
      ok = eval_nodes<M>(P, lamS, Nc, phiL, wL, 1, tid, 256, US, JS, ssum);
      ok = __syncthreads_and(ok);
      if (!ls) {
        accepted = 1;
        break;
      }
      if (ok) {
        double v1[1] = {ssum - (row_live ? lt * uh : 0.0)};
        block_sum<1>(v1, red);
        if (v1[0] <= L0 - 1e-4 * t * slope) {
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
    lam = lt;
    ++its;
    nfresh += stale ? 0 : 1;
    if (!ok) {
      status |= kStRealizability;
      break;
    }
    const double res_old = res;
    res = gradient();
    // a step from the stored inverse must contract the residual by theta, else
    // the inverse is retired (the next iteration, in this or a later step,
    // assembles afresh)
    if (stale && !(res <= P.reuse_theta * res_old)) {
      chord = false;
      if (tid == 0) P.hinv_ok[cell] = 0;
      have_inv = false;
    }
    if (P.one_shot) break;
  }

  // ---- write back: dual, nodal ansatz, wave speeds
  if (row_live) P.lam[gidx] = lam;
  double sx = 0.0, sy = 0.0;
  for (int q = tid; q < Q; q += 256) {
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
  sx = wave_max(sx);
  sy = wave_max(sy);
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6)] = sx;
    red[2 * (tid >> 6) + 1] = sy;
  }
  __syncthreads();
  if (tid == 0) {
    const double mx = nan_max(nan_max(red[0], red[2]), nan_max(red[4], red[6]));
    const double my = nan_max(nan_max(red[1], red[3]), nan_max(red[5], red[7]));
    const int slot = (blk & (kSlots - 1)) * kSlotStride;
    if (P.mode == 0) {
      unsigned long long* bs = P.blk_stats + kBlkStats * static_cast<size_t>(blk);
      bs[0] += static_cast<unsigned long long>(its);
      if (static_cast<unsigned long long>(its) > bs[1]) bs[1] = static_cast<unsigned long long>(its);
      bs[2] += 1ull;
      bs[3] += static_cast<unsigned long long>(nfresh);
      if (status) atomicOr(&P.ctrl->status, status);
      atomicMax(&P.ctrl->amax[P.parity][0][slot], speed_bits(mx));
      if (P.dim == 2) atomicMax(&P.ctrl->amax[P.parity][1][slot], speed_bits(my));
    } else {
      if (status) atomicOr(&P.ctrl->setup_status, status);
      atomicMax(&P.ctrl->amax[0][0][slot], speed_bits(mx));
      if (P.dim == 2) atomicMax(&P.ctrl->amax[0][1][slot], speed_bits(my));
    }
  }
}

// PREC bit 0: BF16-split MFMA Hessian; bit 1: inexact-Hessian Newton.
// Two workgroups per CU up to T = 6 in every variant (the launch is
// occupancy bound; uncapped, the MFMA accumulators of the BF16 variants,
// and at T = 6 the FP64 variants' pending-mode and counter state, push the
// register count just past two wavefronts' share: the FP64 T = 6 kernel
// took 259 registers, one wavefront per SIMD, and ran the 2D bump at 0.57x);
// larger tiles do not fit
template <int M, int T, int PREC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T <= 6 ? 2 : 1)))
void newton_big_kernel(DualParams P) {
  if (P.pend) {  // after the chord kernel: the handed-on cells
    const int n = static_cast<int>(P.ctrl->pend_len[P.parity][P.cls]);
    for (int vb = blockIdx.x; vb < n; vb += gridDim.x) {
      newton_big_body<M, T, PREC>(P, vb);
      __syncthreads();
    }
    return;
  }
  newton_big_body<M, T, PREC>(P, blockIdx.x);
}

template <int M, int T, int PREC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(T <= 6 ? 2 : 1)))
void newton_big_batched(const DualParams* __restrict__ PP,
                                                          const int* __restrict__ begin, int n) {
  const int k = batch_problem(begin, n, blockIdx.x);
  if (PP[k].pend) {
    const DualParams& P = PP[k];
    const int n = static_cast<int>(P.ctrl->pend_len[P.parity][P.cls]);
    for (int vb = blockIdx.x - begin[k]; vb < n; vb += kPendBlocks) {
      newton_big_body<M, T, PREC>(P, vb);
      __syncthreads();
    }
    return;
  }
  newton_big_body<M, T, PREC>(PP[k], blockIdx.x - begin[k]);
}

}  // namespace ipm
