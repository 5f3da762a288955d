// Kinetic flux and moment update (Sec. 3.1 eq:momentIterationFunction in
// the quadrature form eq:momentUpQuadrature; Sec. 3.2), the time step and
// the steady residual eq:residualSteady.
//
// A group of G lanes owns one cell.  Lanes over quadrature nodes read the
// nodal ansatz of the cell and its neighbours (written by the dual kernel),
// apply the deterministic numerical flux per node and form the nodal update
// u - dt/dx (g_r - g_l) [- dt/dy (g_n - g_s)] in LDS; lanes over moments then
// project it on the basis.  The old-moment term is the ansatz h(lambda_c)
// itself, as in eq:momentIterationFunction.
//
// The same kernel takes the tau test of the next time step at its warm
// start: with lambda^n unchanged, the dual gradient is h(lambda^n) - uhat^{n+1}
// = <u_s(lambda^n . phi) phi>_Q - uhat^{n+1}, and both terms are at hand.
// Cells whose residual is clearly below tau (below tau/2, so rounding of
// this shortcut cannot change the outcome of the test) keep their dual and
// nodal ansatz, and their wave speeds enter the next step's slots here;
// the others are appended to the next step's Newton lists.
//
// With dynamic adaptivity (Sec. 5, Alg. ad-IPM) the same pass picks each
// cell's level for the next step from its ansatz and projects the update on
// that level; the step's dual kernels read the levels of their own parity,
// the update writes the other parity's.
//
// Step bookkeeping avoids device-scope fences: every block derives the same
// dt from the 64 speed slots; block 0 alone advances t, the step count and
// the stop flag of the next step parity; the residual is written as one
// partial per block and reduced in fixed order by a one-block kernel.
#pragma once

#include "dual.hpp"

namespace ipm {

// Refinement retardation (Sec. 5, Alg. adosIPM): stage l caps the levels at
// deg[l]; the residual kernel advances the stage when the steady residual
// reaches eps[l].  One per problem in device memory.
constexpr int kMaxRetard = 16;
struct Retard {
  int n, stage;
  int deg[kMaxRetard];
  double eps[kMaxRetard];
};

struct UpdateParams {
  const double* __restrict__ wphi;   // [Q][kp]
  int N, Q, kp, cells, nx, ny, dim;
  const int8_t* __restrict__ cellN;
  const double* __restrict__ nodal;  // [cells][Q][M]
  const double* __restrict__ ghost;  // [4][Q][M] Dirichlet ghost nodal states
  // [cells][M][N] the step's old moments; with gwarm, overwritten by the
  // next step's warm-start dual gradient once read
  double* __restrict__ uold;
  double* __restrict__ s0;           // [cells] next step's <s_*> at the warm start (gwarm), else null
  int gwarm;                         // 1: leave the warm start for the chord kernels (Euler entropy)
  int stage_table;                   // 1: the weighted basis table is staged in LDS (small tables)
  double* __restrict__ unew;         // [cells][M][N]
  double* __restrict__ res_part;     // [gridDim.x]
  int bc[4];
  int flux;
  double gamma, cfl, dx, dy, vol, t_end;
  double tau;
  int one_shot;
  int* lists[kCls];                  // per size class: [64][list_cap] Newton lists of the next step
  int list_cap[kCls];
  StepCtrl* ctrl;
  int parity;
  // dynamic adaptivity (adapt = 1): the next step's level of every cell goes
  // to cellN_next, and a lowered cell's dual loses the modes above its level
  int adapt, p, deg_min, deg_max;
  double delta_lo, delta_hi;
  int8_t* __restrict__ cellN_next;   // [cells] modes of the next step
  double* __restrict__ lam;          // [cells][M][N]
  const Retard* retard;              // null: no level cap
  unsigned cls_map;                  // 4 bits per size class: the class whose lists take its cells
  const double* __restrict__ ctp;    // analytic SG flux: [N][N][N] <phi_i phi_a phi_b> (else null)
  unsigned char* __restrict__ hinv_ok;  // adaptive inexact-Hessian Newton: stored inverses (else null)
};

// index of the neighbour across side 0 (x-) or 1 (x+) of a 1D cell: the
// cell itself at an outflow boundary, wrapped when periodic
__device__ __forceinline__ int neighbour_1d(const UpdateParams& P, int ix, int side) {
  const int j = side == 0 ? ix - 1 : ix + 1;
  if (j >= 0 && j < P.nx) return j;
  return P.bc[side] == kBcPeriodic ? (j + P.nx) % P.nx : ix;
}

// number of basis functions of total degree <= d in p dimensions,
// binomial(d + p, p) (eq:numberBasisFcts); 0 for d = -1
__device__ __forceinline__ int basis_count(int p, int d) {
  int n = 1;
  for (int k = 1; k <= p; ++k) n = n * (d + k) / k;
  return n;
}

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

// largest wave speeds of the step: the first wavefront reads the 64 slots,
// one per lane (step_slots, issued early), and reduces them; the result is
// shared through LDS.
__device__ __forceinline__ void step_slots(const StepCtrl* C, int parity, int dim, double& vx,
                                           double& vy) {
  vx = vy = 0.0;
  if (threadIdx.x < 64) {
    const int s = threadIdx.x;
    vx = __longlong_as_double(static_cast<long long>(C->amax[parity][0][s * kSlotStride]));
    if (dim == 2)
      vy = __longlong_as_double(static_cast<long long>(C->amax[parity][1][s * kSlotStride]));
  }
}

__device__ __forceinline__ void step_speeds(const StepCtrl* C, double vx, double vy, double& ax,
                                            double& ay, double* sh) {
  if (threadIdx.x < 64) {
    vx = wave_max(vx);
    vy = wave_max(vy);
    if (threadIdx.x == 0) {
      sh[0] = nan_max(vx, C->ghost_amax[0]);
      sh[1] = nan_max(vy, C->ghost_amax[1]);
    }
  }
  __syncthreads();
  ax = sh[0];
  ay = sh[1];
}

template <int M, int G>
__device__ __forceinline__ void update_body(const UpdateParams& P, const int blk) {
  StepCtrl* C = P.ctrl;
  // independent loads first, so that their round trips overlap: the stop
  // flags, the step's speed slots, and (below) the tables, this lane's first
  // nodes of the cell and its neighbours and its first old moment
  const int stop_done = C->done[P.parity];
  const unsigned stop_status = C->status;
  double slot_x, slot_y;
  step_slots(C, P.parity, P.dim, slot_x, slot_y);
  extern __shared__ double smem[];
  const int Q = P.Q, kp = P.kp, N = P.N;
  // the weighted basis table: staged in LDS when small, else read from
  // device memory (cached), which leaves the LDS to more wavefronts per CU
  const double* __restrict__ wphiL = P.wphi;
  double* tail = smem;
  if (P.stage_table) {
    for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) smem[k] = P.wphi[k];
    wphiL = smem;
    tail = smem + Q * kp;
  }
  constexpr int CPW = 64 / G;
  const int groups = (blockDim.x >> 6) * CPW;
  const bool analytic = M == 1 && P.flux == kFluxSgAnalytic;
  double* ctpL = tail;                                   // analytic flux: [N][N][N]
  if (analytic)
    for (int k = threadIdx.x; k < N * N * N; k += blockDim.x) ctpL[k] = P.ctp[k];
  double* UT = ctpL + (analytic ? N * N * N : 0);         // per group [Q][M] updated nodes
  double* UC = UT + static_cast<size_t>(groups) * Q * M;  // per group [Q][M] current nodes
  double* red = UC + static_cast<size_t>(groups) * Q * M;

  __shared__ double sh_speed[2];
  __shared__ int s_route[16];
  const int lane = threadIdx.x & 63;
  const int gid = (threadIdx.x >> 6) * CPW + lane / G;
  const int r = lane % G;
  const int cell = blk * groups + gid;
  // operands that do not depend on the time step are requested before the
  // step's speed reduction, so the two memory round trips overlap: this
  // lane's first node of the cell and of its neighbours, and the old moments
  // that this lane's projection replaces first
  const double *uc = nullptr, *uw = nullptr, *ue = nullptr, *us = nullptr, *un = nullptr;
  // small cells on few nodes project one moment (variable, mode) per lane
  // over all nodes: one load and one store per lane instead of M of each
  const bool direct = M * N <= G && Q <= 32;
  double pc[M], pw[M], pe[M], ps[M], pn[M], uoldp[M];
#pragma unroll
  for (int b = 0; b < M; ++b) uoldp[b] = 0.0;
  if (cell < P.cells) {
    const int ix = cell % P.nx, iy = cell / P.nx;
    uc = P.nodal + static_cast<size_t>(cell) * Q * M;
    uw = neighbour_nodal<M>(P, ix, iy, 0);
    ue = neighbour_nodal<M>(P, ix, iy, 1);
    us = P.dim == 2 ? neighbour_nodal<M>(P, ix, iy, 2) : uc;
    un = P.dim == 2 ? neighbour_nodal<M>(P, ix, iy, 3) : uc;
    if (r < Q) {
#pragma unroll
      for (int b = 0; b < M; ++b) {
        pc[b] = uc[r * M + b];
        pw[b] = uw[r * M + b];
        pe[b] = ue[r * M + b];
        ps[b] = us[r * M + b];
        pn[b] = un[r * M + b];
      }
    }
    if (direct) {  // this lane's one moment
      if (r < M * N) uoldp[0] = P.uold[static_cast<size_t>(cell) * M * N + r];
    } else if (r < N) {
#pragma unroll
      for (int b = 0; b < M; ++b) uoldp[b] = P.uold[static_cast<size_t>(cell) * M * N + static_cast<size_t>(b) * N + r];
    }
  }
  if (stop_done || stop_status) {  // uniform: the block leaves before any barrier
    if (blk == 0 && threadIdx.x == 0) {
      C->done[P.parity ^ 1] = 1;
      C->t[P.parity ^ 1] = C->t[P.parity];
    }
    return;
  }
  double ax, ay;
  step_speeds(C, slot_x, slot_y, ax, ay, sh_speed);
  const double t0 = C->t[P.parity];
  double dt = P.dim == 2 ? P.cfl / (ax / P.dx + ay / P.dy) : P.cfl * P.dx / ax;
  bool last = false;
  if (P.t_end > 0.0 && t0 + dt >= P.t_end) {
    dt = P.t_end - t0;
    last = true;
  }
  const double lfx = P.dx / (2.0 * dt), lfy = P.dy / (2.0 * dt);

  double* ut = UT + static_cast<size_t>(gid) * Q * M;
  double* uq = UC + static_cast<size_t>(gid) * Q * M;
  double res_cell = 0.0, nx_speed = 0.0, ny_speed = 0.0;
  int finite = 1, route = 0;
  if (cell < P.cells) {
    const double rx = dt / P.dx, ry = dt / P.dy;
    for (int q = r; q < Q; q += G) {
      double c[M], l[M], rr[M], gl[M], gr[M], acc[M];
      const bool first = q == r;
#pragma unroll
      for (int b = 0; b < M; ++b) {
        c[b] = first ? pc[b] : uc[q * M + b];
        l[b] = first ? pw[b] : uw[q * M + b];
        rr[b] = first ? pe[b] : ue[q * M + b];
      }
      // each state's division and square root once (the cell's own state
      // enters four face fluxes and its wave speeds)
      const FluxState<M> sc = flux_state<M>(P.gamma, c);
      const int kind = analytic ? kFluxLF : P.flux;
      {
        const FluxState<M> sr = flux_state<M>(P.gamma, rr);
        const FluxState<M> sl = flux_state<M>(P.gamma, l);
        numerical_flux_s<M>(kind, 0, c, sc, rr, sr, lfx, gr);
        numerical_flux_s<M>(kind, 0, l, sl, c, sc, lfx, gl);
      }
#pragma unroll
      for (int b = 0; b < M; ++b) acc[b] = c[b] - rx * (gr[b] - gl[b]);
      if (P.dim == 2) {
#pragma unroll
        for (int b = 0; b < M; ++b) {
          l[b] = first ? ps[b] : us[q * M + b];
          rr[b] = first ? pn[b] : un[q * M + b];
        }
        const FluxState<M> sr = flux_state<M>(P.gamma, rr);
        const FluxState<M> sl = flux_state<M>(P.gamma, l);
        numerical_flux_s<M>(P.flux, 1, c, sc, rr, sr, lfy, gr);
        numerical_flux_s<M>(P.flux, 1, l, sl, c, sc, lfy, gl);
#pragma unroll
        for (int b = 0; b < M; ++b) acc[b] -= ry * (gr[b] - gl[b]);
      }
#pragma unroll
      for (int b = 0; b < M; ++b) {
        ut[q * M + b] = acc[b];
        uq[q * M + b] = c[b];
      }
      if (!P.one_shot) {
        double f[M], sx, sy = 0.0;
        state_flux<M>(sc, 0, c, f, sx);
        if (P.dim == 2) state_flux<M>(sc, 1, c, f, sy);
        nx_speed = nan_max(nx_speed, sx);
        ny_speed = nan_max(ny_speed, sy);
      }
    }
    wave_sync();
    const int Nc = P.cellN ? static_cast<int>(P.cellN[cell]) : N;
    // Alg. ad-IPM: the indicator eq:errorIndicator of the first variable of
    // the ansatz at the cell's level d moves the cell one level down or up.
    // The basis is orthonormal, so the averages of the squared truncations
    // are sums of squared ansatz moments (exact for a rule of >= d+1 points
    // per dimension).  The moments below are projected on the new level
    // (eq:adaptiveFVUpdate); a lowered cell drops its dual's top modes and
    // always goes to Newton.
    int Nn = Nc;
    bool lowered = false;
    if (P.adapt) {
      int d = 0;
      while (basis_count(P.p, d) < Nc) ++d;
      const int Nlo = basis_count(P.p, d - 1);
      double top = 0.0, all = 0.0;
      for (int i = r; i < Nc; i += G) {
        double h = 0.0;
        for (int q = 0; q < Q; ++q) h = fma(uq[q * M], wphiL[q * kp + i], h);
        all = fma(h, h, all);
        if (i >= Nlo) top = fma(h, h, top);
      }
      top = group_sum<G>(top);
      all = group_sum<G>(all);
      const double ind = top / all;
      int dn = d;
      if (ind < P.delta_lo && d > P.deg_min) dn = d - 1;
      else if (ind > P.delta_hi && d < P.deg_max) dn = d + 1;
      if (P.retard) dn = min(dn, P.retard->deg[P.retard->stage]);  // Alg. adosIPM cap
      Nn = basis_count(P.p, dn);
      if (r == 0) P.cellN_next[cell] = static_cast<int8_t>(Nn);
      // a stored inverse Hessian belongs to the cell's old level
      if (Nn != Nc && P.hinv_ok != nullptr && r == 0) P.hinv_ok[cell] = 0;
      if (Nn < Nc) {
        lowered = true;
        for (int k = r; k < M * N; k += G) {
          const int i = k % N;
          if (i >= Nn && i < Nc) P.lam[static_cast<size_t>(cell) * M * N + k] = 0.0;
        }
      }
    }
    double d2 = 0.0, gsq[M];
#pragma unroll
    for (int b = 0; b < M; ++b) gsq[b] = 0.0;
    const double* lw = nullptr;
    const double* lc = nullptr;
    const double* le = nullptr;
    if (analytic) {
      const int ix = cell % P.nx;
      lw = P.lam + static_cast<size_t>(neighbour_1d(P, ix, 0)) * N;
      lc = P.lam + static_cast<size_t>(cell) * N;
      le = P.lam + static_cast<size_t>(neighbour_1d(P, ix, 1)) * N;
    }
    if (analytic) {
      for (int k = r; k < M * N; k += G) {
        const int b = k / N, i = k % N;
        double v = 0.0, h = 0.0;
        if (i < Nn)
          for (int q = 0; q < Q; ++q) {
            const double w = wphiL[q * kp + i];
            v = fma(ut[q * M + b], w, v);
            h = fma(uq[q * M + b], w, h);
          }
        if (i < Nn) {
          // App. A, eq:numFluxAnalytic on the duals (quadratic entropy: the
          // dual is the SG moment vector): F_i(u) = u^T C_i u / 2,
          // G = (F(u_l) + F(u_r)) / 2 - dx / (2 dt) (u_r - u_l)
          double fw = 0.0, fc = 0.0, fe = 0.0;
          for (int a = 0; a < N; ++a) {
            const double* Ca = ctpL + (static_cast<size_t>(i) * N + a) * N;
            double sw = 0.0, sc = 0.0, se = 0.0;
            for (int bb = 0; bb < N; ++bb) {
              sw = fma(Ca[bb], lw[bb], sw);
              sc = fma(Ca[bb], lc[bb], sc);
              se = fma(Ca[bb], le[bb], se);
            }
            fw = fma(0.5 * sw, lw[a], fw);
            fc = fma(0.5 * sc, lc[a], fc);
            fe = fma(0.5 * se, le[a], fe);
          }
          const double gr = 0.5 * (fc + fe) - lfx * (le[i] - lc[i]);
          const double gl = 0.5 * (fw + fc) - lfx * (lc[i] - lw[i]);
          v = lc[i] - dt / P.dx * (gr - gl);
        }
        const size_t off = static_cast<size_t>(cell) * M * N + k;
        const double d = v - ((M == 1 && k == r) ? uoldp[0] : P.uold[off]);
        d2 = fma(d, d, d2);
        finite &= (v == v && fabs(v) < 1e300) ? 1 : 0;
        P.unew[off] = v;
        const double g = h - v;  // next step's dual gradient at its warm start
#pragma unroll
        for (int bb = 0; bb < M; ++bb) gsq[bb] += (bb == b) ? g * g : 0.0;
      }
    } else if (direct) {
      // lane r: moment k = r of the cell (variable k / N, mode k mod N)
      for (int k = r; k < M * N; k += G) {
        const int b = k / N, i = k % N;
        double v = 0.0, h = 0.0;
        if (i < Nn)
          for (int q = 0; q < Q; ++q) {
            const double w = wphiL[q * kp + i];
            v = fma(ut[q * M + b], w, v);
            h = fma(uq[q * M + b], w, h);
          }
        const size_t off = static_cast<size_t>(cell) * M * N + k;
        const double d = v - (k == r ? uoldp[0] : P.uold[off]);
        d2 = fma(d, d, d2);
        finite &= (v == v && fabs(v) < 1e300) ? 1 : 0;
        P.unew[off] = v;
        const double g = h - v;  // next step's dual gradient at its warm start
#pragma unroll
        for (int bb = 0; bb < M; ++bb) gsq[bb] += (bb == b) ? g * g : 0.0;
        if (P.gwarm && i < Nn) P.uold[off] = g;
        if (P.gwarm && k == 0) P.s0[cell] = (P.gamma - 1.0) * h;
      }
    } else {
      // projection on the Nn modes of the cell's level: lane r takes mode
      // i = r mod Nn for every variable, over the nodes q = s, s + S, ...
      // of its node group s = r / Nn (S groups, a power of two); the groups
      // are then added pairwise (s takes s + o, o = S/2, ..., 1).  Wide
      // levels (Nn > G) take modes r, r + G, ... over all nodes.
      const bool wide = Nn > G;
      int S = 1;
      if (!wide)
        while (2 * S * Nn <= G) S *= 2;
      int Smax = 1;  // uniform over the wavefront, so every lane joins each exchange
      for (int e = 1; e <= 6; ++e)
        if (__ballot(S >= (1 << e)) != 0ull) Smax = 1 << e;
      const int rounds = wide ? (Nn + G - 1) / G : 1;
      for (int t = 0; t < rounds; ++t) {
        const int i = wide ? r + t * G : r % Nn;
        const int sg = wide ? 0 : r / Nn;
        const bool act = wide ? i < Nn : sg < S;
        double v[M], h[M];
#pragma unroll
        for (int b = 0; b < M; ++b) v[b] = h[b] = 0.0;
        if (act)
          for (int q = sg; q < Q; q += S) {
            const double w = wphiL[q * kp + i];
#pragma unroll
            for (int b = 0; b < M; ++b) {
              v[b] = fma(ut[q * M + b], w, v[b]);
              h[b] = fma(uq[q * M + b], w, h[b]);
            }
          }
        for (int o = Smax >> 1; o >= 1; o >>= 1) {
          const bool take = sg < o && sg + o < S;
          const int src = take ? lane + o * Nn : lane;
#pragma unroll
          for (int b = 0; b < M; ++b) {
            const double pv = __shfl(v[b], src, 64);
            const double ph = __shfl(h[b], src, 64);
            if (take) {
              v[b] += pv;
              h[b] += ph;
            }
          }
        }
        if (act && sg == 0) {
#pragma unroll
          for (int b = 0; b < M; ++b) {
            const size_t off = static_cast<size_t>(cell) * M * N + static_cast<size_t>(b) * N + i;
            // the first round's storing lanes hold mode i = r: prefetched
            const double d = v[b] - (t == 0 ? uoldp[b] : P.uold[off]);
            d2 = fma(d, d, d2);
            finite &= (v[b] == v[b] && fabs(v[b]) < 1e300) ? 1 : 0;
            P.unew[off] = v[b];
            const double g = h[b] - v[b];  // next step's dual gradient at its warm start
            gsq[b] = fma(g, g, gsq[b]);
            if (P.gwarm) P.uold[off] = g;
          }
          // Euler entropy: s_*(lambda . phi) = (gamma - 1) rho, so its
          // quadrature sum is (gamma - 1) times mode 0 of the density's h
          if (P.gwarm && i == 0) P.s0[cell] = (P.gamma - 1.0) * h[0];
        }
      }
      // modes above the level: zero (a lowered cell's old moments there
      // enter the residual).  Without adaptivity a cell's level is fixed
      // and both moment buffers hold zeros there from set-up on.
      const int nz = P.adapt ? N - Nn : 0;
      for (int k = r; k < M * nz; k += G) {
        const size_t off = static_cast<size_t>(cell) * M * N + static_cast<size_t>(k / nz) * N + Nn + k % nz;
        const double d = P.uold[off];
        d2 = fma(d, d, d2);
        P.unew[off] = 0.0;
      }
    }
    d2 = group_sum<G>(d2);
    res_cell = P.vol * sqrt(d2);
    if (!P.one_shot) {
      double resn = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) resn += sqrt(group_sum<G>(gsq[b]));
      // NaN routes to Newton, which reports it; the value is the list class + 1
      route = (resn < 0.5 * P.tau && !lowered)
                  ? 0 : 1 + static_cast<int>((P.cls_map >> (4 * size_class(Nn * M))) & 15u);
    } else if (P.adapt) {  // one-shot: every cell, at its new level
      route = 1 + static_cast<int>((P.cls_map >> (4 * size_class(Nn * M))) & 15u);
    }
  }
  // speeds of the cells whose nodal ansatz carries over to the next step
  nx_speed = route ? 0.0 : nx_speed;
  ny_speed = route ? 0.0 : ny_speed;
  nx_speed = wave_max(nx_speed);
  ny_speed = wave_max(ny_speed);
  finite = __ballot(!finite) == 0ull ? 1 : 0;
  // fixed-order block partial of the residual
  if (r == 0) {
    red[2 * gid] = res_cell;
    red[2 * gid + 1] = finite ? 0.0 : 1.0;
    s_route[gid] = (cell < P.cells) ? route : 0;
  }
  if (lane == 0) {
    red[2 * groups + 2 * (threadIdx.x >> 6)] = nx_speed;
    red[2 * groups + 2 * (threadIdx.x >> 6) + 1] = ny_speed;
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // wavefront 0, all lanes: block totals and list appends
    const int k = threadIdx.x;
    const int rk = k < groups ? s_route[k] : 0;
    const int slot = blk & (kSlots - 1);
    if (k == 0) {
      double sres = 0.0, bad = 0.0;
      for (int g = 0; g < groups; ++g) {
        sres += red[2 * g];
        bad += red[2 * g + 1];
      }
      P.res_part[blk] = sres;
      if (bad > 0.0 || !(ax == ax) || !(ay == ay) || !(dt > 0.0 || last))
        atomicOr(&C->status, kStNonfinite);
      if (!P.one_shot) {
        double mx = 0.0, my = 0.0;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
          mx = nan_max(mx, red[2 * groups + 2 * w]);
          my = nan_max(my, red[2 * groups + 2 * w + 1]);
        }
        atomicMax(&C->amax[P.parity ^ 1][0][slot * kSlotStride], speed_bits(mx));
        if (P.dim == 2) atomicMax(&C->amax[P.parity ^ 1][1][slot * kSlotStride], speed_bits(my));
      }
    }
    if (!P.one_shot || P.adapt)
      for (int c = 0; c < kCls; ++c) {
        // groups routed to class c, in group order: one atomic per class
        const unsigned long long m = __ballot(rk == c + 1);
        if (m == 0ull) continue;  // uniform
        int base = 0;
        if (k == 0)
          base = static_cast<int>(atomicAdd(&C->list_len[list_len_index(P.parity ^ 1, c, slot)],
                                            static_cast<unsigned>(__popcll(m))));
        base = __shfl(base, 0, 64);
        if (rk == c + 1) {
          const int pos = base + __popcll(m & ((1ull << k) - 1ull));
          if (pos < P.list_cap[c])
            P.lists[c][static_cast<size_t>(slot) * P.list_cap[c] + pos] = blk * groups + k;
        }
      }
    if (blk == 0 && k == 0) {
      C->gwarm[P.parity ^ 1] = P.gwarm;
      C->t[P.parity ^ 1] = last ? P.t_end : t0 + dt;
      C->done[P.parity ^ 1] = last ? 1 : 0;
      C->dt_last = dt;
      C->amax_last = P.dim == 2 ? nan_max(ax, ay) : ax;
      C->steps += 1;
    }
  }
}

template <int M, int G>
__global__ __launch_bounds__(256) void update_kernel(UpdateParams P) {
  update_body<M, G>(P, blockIdx.x);
}

template <int M, int G>
__global__ __launch_bounds__(256) void update_batched(const UpdateParams* __restrict__ PP,
                                                      const int* __restrict__ begin, int n) {
  const int k = batch_problem(begin, n, blockIdx.x);
  update_body<M, G>(PP[k], blockIdx.x - begin[k]);
}

#ifdef IPM_HOST_UNIT  // defined once, in the host runtime's unit that launches it
// One block: residual of the last update (fixed summation order) and, for
// steady problems, the stop test eq:residualSteady <= eps.  Also folds the
// per-block Newton counters into the control block when `close` is set.
__global__ __launch_bounds__(256) void residual_kernel(StepCtrl* C, const double* res_part,
                                                       int nparts, double steady_eps, int parity,
                                                       const unsigned long long* blk_stats,
                                                       int nblk, int close, Retard* R) {
  __shared__ double red[256];
  __shared__ unsigned long long rit[256];
  __shared__ unsigned long long rmx[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) s += res_part[k];
  red[threadIdx.x] = s;
  unsigned long long it = 0, mx = 0;
  if (close)
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
      it += blk_stats[kBlkStats * k];
      mx = blk_stats[kBlkStats * k + 1] > mx ? blk_stats[kBlkStats * k + 1] : mx;
    }
  rit[threadIdx.x] = it;
  rmx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      rit[threadIdx.x] += rit[threadIdx.x + w];
      rmx[threadIdx.x] = rmx[threadIdx.x] > rmx[threadIdx.x + w] ? rmx[threadIdx.x]
                                                                  : rmx[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (C->steps > 0) C->residual = red[0];
    // steady stop; with refinement retardation only in the last stage, and
    // before it the stage advances at its own tolerance
    if (!close && !C->done[parity] && !C->status && steady_eps > 0.0 && C->steps > 0) {
      const bool final_stage = !R || R->stage >= R->n - 1;
      if (final_stage) {
        if (red[0] <= steady_eps) C->done[parity ^ 1] = 1;
      } else if (!C->done[parity ^ 1] && red[0] <= R->eps[R->stage]) {
        R->stage += 1;
      }
    }
    if (close) {
      C->newton_iters = rit[0];
      C->max_iters = static_cast<unsigned>(rmx[0]);
    }
  }
}
#endif

}  // namespace ipm
