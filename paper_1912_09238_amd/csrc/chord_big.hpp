// Chord steps of the inexact-Hessian Newton for cells of the workgroup
// kernel (dual_big.hpp: more than 64 unknowns, T x T register tiles).
//
// As on register rows (chord.hpp), a chord iteration needs the ansatz and the
// gradient of eq:L at the nodes, the tau test of eq:tauCrit, the product of
// the stored inverse Hessian with the gradient, and the step-length search;
// here one wavefront runs one cell.  Its lane l stands for the four threads
// l, l + 64, l + 128, l + 192 of the workgroup kernel (as node, as row and as
// tile owner), and every sum is formed as there: per-thread partial sums,
// each wavefront-sum over the same 64 threads, the four combined as
// (w0 + w1) + (w2 + w3); the product with the stored tiles per tile row,
// then over the 16 column threads in ascending order.  The pass over the
// nodes and the stored product are the workgroup kernel's bit for bit; the
// scalar sums of the step (residual, line search, the L-BFGS correction of
// the cell's last accepted step, which the workgroup kernel does not take)
// add a lane's four slots first and take one wavefront sum.  A cell without a valid
// inverse, or whose step fails to contract the dual residual by theta, is
// handed on (hinv_ok = 2) to the workgroup kernel in pending mode.
#pragma once

#include "chord.hpp"
#include "dual_big.hpp"

namespace ipm {

// Secant pairs kept per cell within a launch (0 or 1): the step applies the
// stored inverse with the L-BFGS correction of the cell's last accepted step.
constexpr int kChordBigPairs = 1;

template <int M, int T>
struct ChordBigCfg {
  static constexpr int NPB = 16 * T;
  static constexpr int NJ = M * (M + 1) / 2;
  // per cell: dual [NPB], ansatz [Q][M], gradient [NPB], step [NPB], and the
  // secant pair s, y [2][NPB]
  __host__ __device__ static int cell_doubles(int Q) { return 5 * NPB + Q * M; }
  // node stride of the table, stored mode by mode (odd: lanes of different
  // modes read different banks)
  __host__ __device__ static int qstride(int Q) { return Q | 1; }
  // tables Phi [kl][Q|1] and w [Q], the cells' areas, 2 stats per cell and 2
  // speeds per wavefront
  __host__ __device__ static size_t lds_bytes(int Q, int kl, int waves) {
    return sizeof(double) * (static_cast<size_t>(kl) * qstride(Q) + Q +
                             static_cast<size_t>(waves) * (cell_doubles(Q) + 4));
  }
};

// three wavefronts per SIMD (168 registers) where LDS allows three
// workgroups per CU (up to T = 6 at 125 nodes), except at T = 5; no request
// there and above (their LDS allows two, and a two-wave cap cost the 144-row
// class 9 % of its time).  T = 5 (the 80-row class of the 125-node batch)
// trades the third wavefront for the staged row sums of the product with
// the stored tiles, which do not fit 168 registers (chord launch 7.69 ->
// 7.01 ms); T = 6 keeps three (the 84-row class of the 64-node bump, whose
// ansatz area cannot stage four tiles, ran 19 % slower with two)
template <int T>
constexpr int chord_big_waves() { return (T <= 4 || T == 6) ? 3 : 1; }

// sum over the workgroup kernel's 256 threads, thread 64 s + lane in slot s
// (the four slots of a lane first: one wavefront sum instead of four)
__device__ __forceinline__ double sum4(const double (&x)[4]) {
  return wave_sum((x[0] + x[1]) + (x[2] + x[3]));
}

template <int M, int T>
__device__ __forceinline__ void chord_big_body(const DualParams& P, const int blk) {
  using Cfg = ChordBigCfg<M, T>;
  constexpr int NPB = Cfg::NPB;
  const bool stop = P.mode == 0 && ((P.ctrl->done[P.parity] != 0) | (P.ctrl->status != 0u));
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  int cell = work_cell(P, blk * waves + wave);
  if (stop) return;  // uniform
  if (P.mode == 0 && P.reset_next && blk == 0) reset_next_step(P);
  if (cell >= 0 && P.hinv_ok[cell] != 1) {
    if (lane == 0) hand_on(P, cell);
    cell = -1;
  }
  if (!__syncthreads_or(cell >= 0)) return;

  const int Q = P.Q, kg = P.kp, kp = P.kl, N = P.N;
  extern __shared__ double smem[];
  const int QT = Cfg::qstride(Q);
  double* phiT = smem;            // [kp][QT]: phi_i(q)
  double* wL = phiT + kp * QT;    // [Q]
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x)
    phiT[(k % kp) * QT + k / kp] = P.phi[(k / kp) * kg + k % kp];
  for (int q = threadIdx.x; q < Q; q += blockDim.x) wL[q] = P.wphi[static_cast<size_t>(q) * kg];
  double* lamS = wL + Q + static_cast<size_t>(wave) * (Cfg::cell_doubles(Q) + 4);
  double* US = lamS + NPB;   // [Q][M]
  double* gS = US + Q * M;   // [NPB]
  double* dS = gS + NPB;     // [NPB]
  double* sP = dS + NPB;     // [NPB] secant pair: s = lambda_k+1 - lambda_k
  double* yP = sP + NPB;     // [NPB]                y = g_k+1 - g_k
  double* stats = yP + NPB;  // [4]: its + listed, status, speeds x, y
  __syncthreads();

  int its = 0, evals = 0;  // evals: passes over the nodes (entry and each trial)
  unsigned status = 0;
  bool pending = false;
  double sx = 0.0, sy = 0.0;
  if (cell >= 0) {
    const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
    const int nc = Nc * M;
    // the four stand-in threads v = lane + 64 s: unknown v (row), node v
    bool live[4];
    int ri[4], ra[4];
    size_t gidx[4];
    double lam[4], uh[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int v = lane + 64 * s;
      live[s] = v < nc;
      ri[s] = v / M;
      ra[s] = v % M;
      gidx[s] = static_cast<size_t>(cell) * M * N + static_cast<size_t>(ra[s]) * N + ri[s];
      lam[s] = live[s] ? P.lam[gidx[s]] : 0.0;
      uh[s] = live[s] ? P.uhat[gidx[s]] : 0.0;
      if (v < NPB) lamS[v] = live[s] ? lam[s] : 0.0;
    }
    const global_fptr Hc =
        (global_fptr)(P.hinv + static_cast<size_t>(P.hinv_slot ? P.hinv_slot[cell] : cell) * P.hinv_stride);
    wave_sync();
    double ssum[4];
    // the ansatz at node v of each stand-in thread: w_q u_s to LDS (the
    // product the gradient sum takes, formed once per node), <s_*> shares
    auto eval = [&]() -> int {
      ++evals;
      int okp = 1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ssum[s] = 0.0;
        const int q = lane + 64 * s;
        if (q < Q) {
          double u[M], ss;
          okp &= node_ansatz<M>(P, lamS, Nc, phiT + q, QT, u, ss) ? 1 : 0;
#pragma unroll
          for (int a = 0; a < M; ++a) US[q * M + a] = u[a] * wL[q];
          ssum[s] = fma(wL[q], ss, ssum[s]);
        }
      }
      wave_sync();
      return __ballot(!okp) == 0ull ? 1 : 0;
    };
    double g[4];
    // the tau residual from the squared gradient entries by variable; with
    // four variables every slot of a lane holds the same variable (64 s +
    // lane = lane mod 4), so one class sum over the lanes serves
    auto residual = [&](const double (&e2)[M][4]) -> double {
      if constexpr (M == 4) {
        double e = 0.0;  // the other variables' entries of a lane are zero
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int b = 0; b < M; ++b) e += e2[b][s];
        return tau_residual4_sq<64>(e);
      }
      double res = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) res += sqrt(sum4(e2[b]));
      return res;
    };
    auto gradient = [&]() -> double {
      double e2[M][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double gg = 0.0;
        if (live[s]) {
          const double* pr = phiT + ri[s] * QT;
          for (int q = 0; q < Q; ++q) gg = fma(US[q * M + ra[s]], pr[q], gg);
          gg -= uh[s];
        }
        g[s] = gg;
#pragma unroll
        for (int b = 0; b < M; ++b) e2[b][s] = (live[s] && ra[s] == b) ? gg * gg : 0.0;
      }
      return residual(e2);
    };
    // the previous update's warm start (Euler entropy): the gradient and
    // <s_*> at this dual, which spares the entry pass over the nodes
    const bool warm = P.gwarm != nullptr && P.ctrl->gwarm[P.parity] != 0;  // uniform
    bool entry_warm = warm;
    double s0 = 0.0;
    int ok = 1;
    double res = 0.0;
    if (warm) {
      double e2[M][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        g[s] = live[s] ? P.gwarm[gidx[s]] : 0.0;
#pragma unroll
        for (int b = 0; b < M; ++b) e2[b][s] = (live[s] && ra[s] == b) ? g[s] * g[s] : 0.0;
      }
      res = residual(e2);
      s0 = P.s0[cell];
    } else {
      ok = eval();
      if (ok) res = gradient();
      else status |= kStRealizability;
    }
    double rho1 = 0.0, alpha = 0.0;  // 1 / (y . s) of the pair; its first-loop coefficient
    bool pair = false;               // uniform
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
      // ---- d = H^-1 g from the stored tiles: tile thread u = 64 s + lane
      // (rows tr + 16 i, columns tc + 16 j) forms its row sums, the 16
      // column threads of a row are then added in ascending order
      // with a secant pair, the stored inverse acts on q = g - alpha y,
      // alpha = rho s . g (the two-loop recursion with one pair)
      if (kChordBigPairs > 0 && pair) {
        double x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int v = lane + 64 * s;
          x[s] = (live[s] && v < NPB) ? sP[v] * g[s] : 0.0;
        }
        alpha = rho1 * sum4(x);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int v = lane + 64 * s;
        if (v < NPB) gS[v] = live[s] ? (pair ? fma(-alpha, yP[v], g[s]) : g[s]) : 0.0;
      }
      wave_sync();
      const int tc = lane & 15;
      double gc[T];
#pragma unroll
      for (int j = 0; j < T; ++j) gc[j] = gS[tc + 16 * j];
      // all 256 tile threads (tile rows tr = 0..15 at every T).  When the
      // ansatz area (free until the next pass over the nodes) holds them,
      // the row sums of IB tiles are formed with all their loads in flight
      // and staged there (rows of 16 at a stride of 17 doubles: the reads
      // below hit distinct banks); one lane per (tile, row) then adds the
      // 16 column sums in ascending order, the order of the broadcast chain
      // of the other path, so both give the same bits.  Only for the tiles
      // outside the three-wavefront register budget: within it the staged
      // form spills (measured 49 % slower at T = 5).
      constexpr int IB = T < 4 ? T : 4;
      constexpr bool staged = chord_big_waves<T>() != 3;
      if (staged && Q * M >= 68 * IB) {  // uniform
        const int rr0 = lane >> 4;
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
          const int u = 64 * s + lane;
#pragma unroll
          for (int i0 = 0; i0 < T; i0 += IB) {
#pragma unroll
            for (int k = 0; k < IB; ++k) {
              const int i = i0 + k;
              if (i < T) {
                double ps = 0.0;
#pragma unroll
                for (int j = 0; j < T; ++j)
                  ps = fma(static_cast<double>(Hc[(i * T + j) * 256 + u]), gc[j], ps);
                US[k * 68 + rr0 * 17 + tc] = ps;
              }
            }
            wave_sync();
            if (lane < 4 * IB) {
              const int k = lane >> 2, rr = lane & 3;
              if (i0 + k < T) {
                const double* pp = US + k * 68 + rr * 17;
                double dv = 0.0;
#pragma unroll
                for (int c = 0; c < 16; ++c) dv += pp[c];
                dS[4 * s + rr + 16 * (i0 + k)] = dv;
              }
            }
            wave_sync();
          }
        }
      } else {
#pragma unroll 1
        for (int s = 0; s < 4; ++s) {
          const int u = 64 * s + lane, tr = u >> 4;
#pragma unroll 1
          for (int i = 0; i < T; ++i) {
            double ps = 0.0;
#pragma unroll
            for (int j = 0; j < T; ++j) ps = fma(static_cast<double>(Hc[(i * T + j) * 256 + u]), gc[j], ps);
            double dv = 0.0;
            dv += row_bcast<0>(ps);
            dv += row_bcast<1>(ps);
            dv += row_bcast<2>(ps);
            dv += row_bcast<3>(ps);
            dv += row_bcast<4>(ps);
            dv += row_bcast<5>(ps);
            dv += row_bcast<6>(ps);
            dv += row_bcast<7>(ps);
            dv += row_bcast<8>(ps);
            dv += row_bcast<9>(ps);
            dv += row_bcast<10>(ps);
            dv += row_bcast<11>(ps);
            dv += row_bcast<12>(ps);
            dv += row_bcast<13>(ps);
            dv += row_bcast<14>(ps);
            dv += row_bcast<15>(ps);
            if (tc == 0) dS[tr + 16 * i] = dv;
          }
        }
      }
      wave_sync();
      double d[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int v = lane + 64 * s;
        d[s] = (live[s] && v < NPB) ? dS[v] : 0.0;
      }
      wave_sync();
      if (kChordBigPairs > 0 && pair) {  // second loop: d += s (alpha - rho y . d)
        double x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int v = lane + 64 * s;
          x[s] = (live[s] && v < NPB) ? yP[v] * d[s] : 0.0;
        }
        const double beta = rho1 * sum4(x);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int v = lane + 64 * s;
          if (live[s] && v < NPB) d[s] = fma(sP[v], alpha - beta, d[s]);
        }
      }
      // ---- step length
      const bool ls = !P.one_shot && res > 1e-6;
      double L0 = 0.0, slope = 0.0;
      if (ls) {
        double x0[4], x1[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          x0[s] = (entry_warm ? 0.0 : ssum[s]) - (live[s] ? lam[s] * uh[s] : 0.0);
          x1[s] = live[s] ? g[s] * d[s] : 0.0;
        }
        L0 = sum4(x0);
        if (entry_warm) L0 += s0;
        slope = sum4(x1);
      }
      entry_warm = false;  // from here on ssum is the accepted trial's
      double t = 1.0, lt[4];
      int accepted = 0;
#pragma unroll 1
      for (int h = 0; h <= 60; ++h) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          lt[s] = lam[s] - t * d[s];
          const int v = lane + 64 * s;
          if (v < NPB) lamS[v] = live[s] ? lt[s] : 0.0;
        }
        wave_sync();
        ok = eval();
        if (!ls) {
          accepted = 1;
          break;
        }
        if (ok) {
          double x[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) x[s] = ssum[s] - (live[s] ? lt[s] * uh[s] : 0.0);
          if (sum4(x) <= L0 - 1e-4 * t * slope) {
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
      if (kChordBigPairs > 0) {  // the new pair (each lane its own entries)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int v = lane + 64 * s;
          if (v < NPB) {
            sP[v] = live[s] ? lt[s] - lam[s] : 0.0;
            yP[v] = live[s] ? -g[s] : 0.0;
          }
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) lam[s] = lt[s];
      ++its;
      if (!ok) {
        status |= kStRealizability;
        break;
      }
      const double res_old = res;
      res = gradient();
      if (kChordBigPairs > 0) {
        double x[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int v = lane + 64 * s;
          x[s] = 0.0;
          if (v < NPB) {
            const double y = live[s] ? yP[v] + g[s] : 0.0;
            yP[v] = y;
            x[s] = sP[v] * y;
          }
        }
        const double ys = sum4(x);
        pair = ys > 0.0;  // strictly convex L: always, up to rounding
        rho1 = pair ? 1.0 / ys : 0.0;
      }
      if (!(res <= P.reuse_theta * res_old)) {
        if (P.one_shot) {
          if (lane == 0) P.hinv_ok[cell] = 0;
        } else {
          pending = true;
        }
        break;
      }
      if (P.one_shot) break;
    }
    // ---- write back: the dual; unless handed on, the nodal ansatz and speeds
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (live[s]) P.lam[gidx[s]] = lam[s];
    if (pending || status) {
      if (lane == 0 && pending) hand_on(P, cell);
    } else {
      // the ansatz of the final dual (staged in lamS), node by node
      for (int q = lane; q < Q; q += 64) {
        double u[M], ss;
        (void)node_ansatz<M>(P, lamS, Nc, phiT + q, QT, u, ss);
#pragma unroll
        for (int b = 0; b < M; ++b) P.nodal[(static_cast<size_t>(cell) * Q + q) * M + b] = u[b];
        double ax, ay;
        wave_speeds<M>(P.cp.gamma, P.dim, u, ax, ay);
        sx = nan_max(sx, ax);
        sy = nan_max(sy, ay);
      }
    }
  }

  // ---- per-block statistics and speed slots
  sx = wave_max(sx);
  sy = wave_max(sy);
  if (lane == 0) {
    stats[0] = pack_stats(its, evals, cell >= 0);
    stats[1] = static_cast<double>(status);
    stats[2] = sx;
    stats[3] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum_its = 0, max_its = 0, listed = 0, sum_evals = 0;
    unsigned st = 0;
    double mx = 0.0, my = 0.0;
    for (int w = 0; w < waves; ++w) {
      const double* o = wL + Q + static_cast<size_t>(w) * (Cfg::cell_doubles(Q) + 4) + Cfg::cell_doubles(Q);
      const unsigned long long v = static_cast<unsigned long long>(o[0]);
      const unsigned long long it = v & 1023ull;
      sum_its += it;
      max_its = it > max_its ? it : max_its;
      sum_evals += (v >> 10) & 0x3fffffffull;
      listed += v >> 40;
      st |= static_cast<unsigned>(o[1]);
      mx = nan_max(mx, o[2]);
      my = nan_max(my, o[3]);
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

template <int M, int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(chord_big_waves<T>())))
void newton_chord_big_kernel(DualParams P) {
  chord_big_body<M, T>(P, blockIdx.x);
}

template <int M, int T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(chord_big_waves<T>())))
void newton_chord_big_batched(const DualParams* __restrict__ PP, const int* __restrict__ begin, int n) {
  const int k = batch_problem(begin, n, blockIdx.x);
  chord_big_body<M, T>(PP[k], blockIdx.x - begin[k]);
}

}  // namespace ipm
