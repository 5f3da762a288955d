// Per-cell dual solve (Sec. 3.1: eq:L, eq:dualIterationFunction,
// eq:tauCrit; one-shot: eq:oneshotIPMdual), n = m*N <= 64 unknowns.
//
// The tau test at the warm start of a time step is taken by the flux-update
// kernel of the previous step (it holds h(lambda) and the new moments), which
// lists the cells that need Newton steps in 64 lists; the other cells keep
// their dual and nodal ansatz unchanged, exactly as a solve that stops at
// iteration 0 would.
//  * newton_kernel: one group of NP lanes per listed cell (NP = n rounded up
//    to 8, 16, 32 or 64; or per cell in one-shot and setup runs) iterates
//    Newton to tau:
//      - unknowns interleaved r = i*m + a (mode i, variable a), so a lower
//        degree is a prefix;
//      - ansatz: lanes over nodes, u_s and the packed grad u_s to LDS;
//      - gradient and the tau test on sum_a |g_a|_2, FP64, reductions on
//        the DPP network;
//      - Hessian H[(i,a)][(k,b)] = sum_q w_q J_q[a][b] phi_i phi_k: lane r
//        accumulates row r in registers;
//      - H d = g: Gauss-Jordan elimination without pivoting (H is SPD).
//        Rows and columns beyond the cell's n unknowns are an identity
//        block.  At each step every row needs the pivot column (16 and 32
//        lanes: DPP row broadcasts plus a 16-lane row swap, register to
//        register; 8 and 64 lanes: through LDS); by symmetry of the Schur
//        complement this column is also the pivot row, so every row is
//        updated from it, the right-hand side is eliminated along, and no
//        back-substitution (no transposed access) is needed;
//      - step length: Armijo backtracking on L when the dual residual
//        exceeds 1e-6, else the full step; one-shot: one full step;
//      - inexact-Hessian variant (PREC bit 1; the outlook of Sec. 7 on not
//        recomputing the Hessian): a fresh Hessian is inverted in place by
//        the symmetric sweep (the matrix stays symmetric, so the broadcast
//        pivot column again serves as the pivot row), the cell's n x n
//        block of -H^-1 goes to HBM, and later iterations of the cell, in
//        this and following steps, take d = H_old^-1 g from it while each
//        such step contracts the dual residual by a factor theta; otherwise
//        the inverse is retired and the next iteration (one-shot: of the
//        next pseudo-time step) assembles and inverts afresh.  The tau test
//        is unchanged;
//      - single-chunk variant (PREC bit 2): for rules of at most NP nodes,
//        which a cell's lanes hold in one chunk; the streaming code is
//        compiled out (fewer registers, a plain node loop).
// The dual, the nodal ansatz (read by the flux update) and the wave speeds
// leave the kernels; the exact variant's Hessian never touches HBM.
// Statistics go to per-block cumulative counters (plain stores) and to 64
// atomic speed slots on separate cache lines; no device-scope fence is
// issued.
#pragma once

#include <type_traits>

#include "device_common.hpp"

namespace ipm {

constexpr int kSlots = 64;
constexpr int kSlotStride = 16;  // 128-byte spacing of atomic slots
// Newton size classes of a cell with n unknowns: groups of 8, 16, 32, 64
// lanes (n <= 64), or the workgroup-per-cell kernel with 16 T x 16 T tiles,
// T = 5, 6, 8, 9 (n <= 80, 96, 128, 144)
constexpr int kCls = 8;
__host__ __device__ inline int size_class(int n) {
  return n > 128 ? 7 : n > 96 ? 6 : n > 80 ? 5 : n > 64 ? 4 : n > 32 ? 3 : n > 16 ? 2 : n > 8 ? 1 : 0;
}
__host__ __device__ inline int class_tiles(int c) { return c == 4 ? 5 : c == 5 ? 6 : c == 6 ? 8 : 9; }

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
  // [parity][class][slot * kSlotStride] lengths of the 64 lists per size
  // class of cells that need Newton steps
  unsigned int list_len[2 * kCls * kSlots * kSlotStride];
  // [parity][class] cells the chord kernels handed on to the full kernel
  unsigned int pend_len[2][kCls];
  // [parity] 1: the update before the step of this parity left the warm-start
  // gradient and <s_*> of every cell (the chord kernels start from them)
  int gwarm[2];
};

__host__ __device__ inline size_t list_len_index(int parity, int cls, int slot) {
  return (static_cast<size_t>(parity) * kCls + cls) * kSlots * kSlotStride +
         static_cast<size_t>(slot) * kSlotStride;
}

// Counters per Newton block (cumulative over steps).
constexpr int kBlkStats = 4;
// Pending mode (after a chord kernel): a launch of this many blocks per
// problem walks the class's list of handed-on cells.
constexpr int kPendBlocks = 32;

struct DualParams {
  const double* __restrict__ phi;   // [Q][kp] Phi, zero padded to kp columns
  const double* __restrict__ wphi;  // [Q][kp] w_q Phi (column 0 holds w_q)
  int N, Q, kp, cells;
  int kl;                           // Phi columns staged in LDS for this launch's class (<= kp)
  int pend;                         // full kernel after the chord kernel: pending cells only
  int* __restrict__ pend_list;      // [class cells] cells handed on (chord kernels append)
  const int8_t* __restrict__ cellN; // modes per cell, or null (all N)
  const double* __restrict__ uhat;  // [cells][M][N]
  // warm start left by the previous update (chord kernels; null: none):
  // the dual gradient at the cell's current dual [cells][M][N] and the
  // quadrature sum of s_* there [cells], valid when ctrl->gwarm[parity]
  const double* __restrict__ gwarm;
  const double* __restrict__ s0;
  double* __restrict__ lam;         // [cells][M][N], in/out
  double* __restrict__ nodal;       // [cells][Q][M], out
  // [gridDim.x][kBlkStats]: Newton iterations, their max over the block's
  // cells, cells the block solved (listed), iterations with a fresh Hessian
  unsigned long long* __restrict__ blk_stats;
  ClosureParams cp;
  double tau;
  int max_newton, one_shot;
  int mode;                         // 0: time step, 1: setup (converge only)
  int dim;
  StepCtrl* ctrl;
  int parity;
  int* __restrict__ lists;          // [64][list_cap] cells of this class needing Newton steps
  int list_cap;                     // 0: cells from `order` (or 0..cells-1 if null)
  int cls;                          // size class of the launch
  int reset_next;                   // block 0 clears the next step's lists and speed slots
  const int* __restrict__ order;    // [order_len] cells of this class, ascending
  int order_len;
  int bcache;                       // precision form: B fragments cached in LDS
  // inexact-Hessian Newton: per cell the inverse Hessian of its last fresh
  // assembly (workgroup kernel: [T*T][256] tiles; small kernel: the cell's
  // nc x nc block of -H^-1 by column, dense), and a valid flag; null: exact
  // Newton.
  // Stored in FP32: a stale inverse only sets the direction of a step whose
  // gradient and tau test stay FP64, and the steps are checked to contract.
  float* __restrict__ hinv;
  unsigned char* __restrict__ hinv_ok;      // [cells]
  long long hinv_stride;                    // floats per cell in hinv
  const int* __restrict__ hinv_slot;        // [cells] slot in hinv (null: the cell index)
  double reuse_theta;                       // a stale step must give res_new <= theta res_old
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

// Broadcast lane N of each 16-lane row to the whole row (64-bit row_newbcast DPP).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  const long long x = __builtin_amdgcn_update_dpp(0ll, __builtin_bit_cast(long long, v), 0x150 + N,
                                                  0xF, 0xF, true);
  return __builtin_bit_cast(double, x);
}

// acc += (lane N of this 16-lane row's src) * mul, one instruction: the
// row_newbcast DPP operand of v_fmac_f64.  Pure ALU; the caller separates it
// from the VALU write of src by at least two wait states (see dpp_guard).
template <int N>
__device__ __forceinline__ void fmac_row_bcast(double& acc, double src, double mul) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
               : "+v"(acc)
               : "v"(src), "v"(mul), "i"(N));
}
// Two wait states between the VALU writes of a and b and the DPP reads that
// follow: a and b are inputs, so their producers are scheduled before it.
__device__ __forceinline__ void dpp_guard(double a, double b) {
  asm volatile("s_nop 1" : : "v"(a), "v"(b));
}

// For aligned 32-lane groups: lo holds the group's lanes 0..15 in both of its
// 16-lane rows, hi its lanes 16..31 (v_permlane16_swap on each 32-bit half).
__device__ __forceinline__ void group32_halves(double v, double& lo, double& hi) {
  const int a = __double2loint(v), b = __double2hiint(v);
  const auto pa = __builtin_amdgcn_permlane16_swap(a, a, false, false);
  const auto pb = __builtin_amdgcn_permlane16_swap(b, b, false, false);
  lo = __hiloint2double(pb[0], pa[0]);
  hi = __hiloint2double(pb[1], pa[1]);
}

// Compile-time loop: f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
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

// 1/x with one Newton step (relative error about 2e-15): the elimination
// multipliers of the register-row solve, where the reciprocal sits on every
// pivot step's dependency chain; the dual update itself stays exact to
// rounding through the final division by the pivots (recip)
__device__ __forceinline__ double recip1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
}

// Ansatz at the nodes q = q0, q0 + step, ... of one cell for the dual lamS
// (interleaved, first Nc modes).  Writes u and packed J to LDS slot q - qoff,
// adds the lane's share of <s_*> to ssum.  Returns the admissible flag.
template <int M>
__device__ __forceinline__ int eval_nodes(const DualParams& P, const double* lamS, int Nc,
                                          const double* phiL, const double* wq, int wstride,
                                          int q0, int step, double* US, double* JS,
                                          double& ssum, int qoff = 0) {
  constexpr int NJ = M * (M + 1) / 2;
  int ok = 1;
#pragma unroll 1
  for (int q = q0; q < P.Q; q += step) {
    double L[M];
#pragma unroll
    for (int a = 0; a < M; ++a) L[a] = 0.0;
    const double* ph = phiL + q * P.kl;
#pragma unroll 4
    for (int i = 0; i < Nc; ++i) {
      const double f = ph[i];
#pragma unroll
      for (int a = 0; a < M; ++a) L[a] = fma(lamS[i * M + a], f, L[a]);
    }
    double u[M], J[NJ], ss;
    ok &= closure<M>(P.cp, L, u, J, ss) ? 1 : 0;
#pragma unroll
    for (int a = 0; a < M; ++a) US[(q - qoff) * M + a] = u[a];
#pragma unroll
    for (int k = 0; k < NJ; ++k) JS[(q - qoff) * NJ + k] = J[k];
    ssum = fma(wq[q * wstride], ss, ssum);
  }
  return ok;
}

// ---------------------------------------------------------------- Newton

// Layout: a group of G = NP / R lanes owns one cell, 64 / G cells per
// wavefront, up to four wavefronts per block.  Lane r of a group holds the R
// Hessian rows r, r + G, ... (all NP columns each) and the matching unknowns;
// R = 1 (one row per lane) in every configuration built.
// Control flow is uniform within a group; groups of one wavefront may leave
// the Newton loop at different iterations (cross-lane operations stay inside
// the group).
template <int M, int NP>
struct NewtonCfg {
  // NP = 16, 32: the elimination broadcasts pivot columns register to
  // register (DPP row broadcast, plus a 16-lane row swap for 32-lane
  // groups); otherwise through LDS.
  static constexpr bool kDpp = (NP == 16 || NP == 32);
  static constexpr int R = 1;
  static constexpr int G = NP / R;
  static constexpr int CPW = 64 / G;
  static constexpr int NJ = M * (M + 1) / 2;
  static constexpr int KCOL = (NP + M - 1) / M;  // table columns the rows read

  // nodes held per group at a time: one per lane (a cell's nodes stream
  // through in chunks), all of them when there are fewer
  __host__ __device__ static int chunk(int Q) { return Q < G ? Q : G; }
  __host__ __device__ static int group_doubles(int Q) {
    return NP + chunk(Q) * (M + NJ) + (kDpp ? 0 : 2 * NP + 2 + NP);
  }
  __host__ __device__ static size_t lds_bytes(int Q, int kp, int waves) {
    // tables, per-group work areas, then 2 stats per group + 2 speeds per wave
    return sizeof(double) * (2 * static_cast<size_t>(Q) * kp +
                             static_cast<size_t>(waves) * CPW * group_doubles(Q) +
                             2 * static_cast<size_t>(waves) * (CPW + 1));
  }
};

// Read-only table through the scalar unit: the basis values of one node are
// the same for every lane, so they need not occupy LDS bandwidth.
typedef const __attribute__((address_space(4))) double* const_dptr;
// Device memory read through the vector memory path (global loads: unlike
// flat loads they do not hold up the wait for LDS results).
typedef const __attribute__((address_space(1))) float* global_fptr;

// The cell of work item `item`: the 64 lists of the launch's size class laid
// end to end (a prefix sum over their lengths, so the listed cells occupy the
// first items of the grid whatever their spread over the lists), or the
// class's cells in ascending order.  Called by every thread of the block.
__device__ __forceinline__ int work_cell(const DualParams& P, int item) {
  if (P.pend) {  // the cells the chord kernel of this step handed on
    const int n = static_cast<int>(P.ctrl->pend_len[P.parity][P.cls]);
    return item < n ? P.pend_list[item] : -1;
  }
  if (P.list_cap > 0) {
    __shared__ int pre[kSlots + 1];
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      int v = min(static_cast<int>(P.ctrl->list_len[list_len_index(P.parity, P.cls, lane)]),
                  P.list_cap);
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
      }
      pre[lane + 1] = v;
      if (lane == 0) pre[0] = 0;
    }
    __syncthreads();
    if (item >= pre[kSlots]) return -1;
    int lo = 0, hi = kSlots - 1;  // the list holding the item: last s with pre[s] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    return P.lists[static_cast<size_t>(lo) * P.list_cap + (item - pre[lo])];
  }
  if (P.order) return item < P.order_len ? P.order[item] : -1;
  return item < P.cells ? item : -1;
}

__device__ __forceinline__ void reset_next_ctrl(StepCtrl* C, int parity) {
  for (int k = threadIdx.x; k < kSlots; k += blockDim.x) {
    C->amax[parity ^ 1][0][k * kSlotStride] = 0ull;
    C->amax[parity ^ 1][1][k * kSlotStride] = 0ull;
  }
  for (int k = threadIdx.x; k < kCls * kSlots; k += blockDim.x)
    C->list_len[list_len_index(parity ^ 1, k / kSlots, k % kSlots)] = 0u;
  for (int k = threadIdx.x; k < kCls; k += blockDim.x) C->pend_len[parity ^ 1][k] = 0u;
}
__device__ __forceinline__ void reset_next_step(const DualParams& P) { reset_next_ctrl(P.ctrl, P.parity); }

template <int M, int NP, int PREC = 0>
__device__ __forceinline__ void newton_body(const DualParams& P, const int blk) {
  using Cfg = NewtonCfg<M, NP>;
  constexpr int G = Cfg::G, CPW = Cfg::CPW, NJ = Cfg::NJ, R = Cfg::R;
  constexpr bool kDpp = Cfg::kDpp;
  // the stop flags are read with the list lengths (one round trip, not two);
  // a stopped problem's block leaves right after, before any write
  const bool stop = P.mode == 0 && ((P.ctrl->done[P.parity] != 0) | (P.ctrl->status != 0u));
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G;
  const int r = lane % G;
  int cell = work_cell(P, (blk * waves + wave) * CPW + grp);
  if (stop) return;  // uniform
  // the flux update of this step fills the next step's speed slots and lists
  if (P.mode == 0 && P.reset_next && blk == 0) reset_next_step(P);
  if (!__syncthreads_or(cell >= 0)) return;

  // kp: LDS stride of the staged table (the class's columns), kg: the
  // global table's
  const int Q = P.Q, kg = P.kp, kp = P.kl, N = P.N;
  // the cell's dual and moments are requested before the tables are staged,
  // so the two memory round trips overlap; unknown (i, a) of row
  // ro = i * M + a; rows r + s * G of this lane
  const int Nc = cell >= 0 ? (P.cellN ? static_cast<int>(P.cellN[cell]) : N) : 0;
  const int nc = Nc * M;
  int ro[R], ii[R], aa[R];
  bool live[R];
  size_t gidx[R];
  double lam[R], uh[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    ro[s] = r + s * G;
    ii[s] = ro[s] / M;
    aa[s] = ro[s] % M;
    live[s] = ro[s] < nc;
    gidx[s] = static_cast<size_t>(cell >= 0 ? cell : 0) * M * N + static_cast<size_t>(aa[s]) * N + ii[s];
    lam[s] = live[s] ? P.lam[gidx[s]] : 0.0;
    uh[s] = live[s] ? P.uhat[gidx[s]] : 0.0;
  }
  extern __shared__ double smem[];
  double* phiL = smem;
  double* wphiL = phiL + Q * kp;
  // the LDS stride is odd (a lane per node reads its own row without bank
  // conflicts) and may exceed the global one by a zero column
  for (int k = threadIdx.x; k < Q * kp; k += blockDim.x) {
    const int i = k % kp;
    const int g = (k / kp) * kg + i;
    phiL[k] = i < kg ? P.phi[g] : 0.0;
    wphiL[k] = i < kg ? P.wphi[g] : 0.0;
  }
  const const_dptr phiC = (const_dptr)(P.phi);
  const int gidx_l = wave * CPW + grp;
  double* lamS = wphiL + Q * kp + static_cast<size_t>(gidx_l) * Cfg::group_doubles(Q);  // [NP]
  const int CH = Cfg::chunk(Q);   // nodes per chunk
  // the chunk holds every node: no re-evaluation (the single-chunk variant
  // is launched only for Q <= NP)
  const bool one_chunk = (PREC & 4) != 0 ? true : CH == Q;
  double* US = lamS + NP;         // [CH][M]
  double* JS = US + CH * M;       // [CH][NJ]
  double* cA = JS + CH * NJ;      // [2][NP] pivot column (LDS elimination)
  double* cX = cA + 2 * NP;       // [2] pivot row's right-hand side
  double* cP = cX + 2;            // [NP] pivots
  double* stats = wphiL + Q * kp + static_cast<size_t>(waves) * CPW * Cfg::group_doubles(Q);
  __syncthreads();

  // elimination steps the wavefront runs: the largest unknown count of its
  // cells (wave-uniform, so each step is a scalar branch; smaller cells see
  // only identity rows in the extra steps)
  const int kmax =
      __builtin_amdgcn_readfirstlane(static_cast<int>(wave_max(static_cast<double>(nc))));
  (void)kmax;

  int its = 0, nfresh = 0;
  unsigned status = 0;
  double sx = 0.0, sy = 0.0;
  if (cell >= 0) {
#pragma unroll
    for (int s = 0; s < R; ++s) lamS[ro[s]] = lam[s];
    wave_sync();
    double ssum = 0.0;
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (grp * G));
    auto group_all = [&](int v) -> int { return (__ballot(!v) & gmask) == 0ull ? 1 : 0; };
    // One pass over the nodes for the dual in lamS, chunk by chunk (lane r:
    // node c0 + r): the ansatz, <s_*> (ssum) and the gradient sums of the
    // lane's rows, node by node in ascending order.  The last chunk stays
    // in US / JS.
    double gacc[R];
    auto grad_pass = [&]() -> int {
      int okp = 1;
      ssum = 0.0;
#pragma unroll
      for (int s = 0; s < R; ++s) gacc[s] = 0.0;
      for (int c0 = 0; c0 < Q; c0 += CH) {
        okp &= eval_nodes<M>(P, lamS, Nc, phiL, wphiL, kp, c0 + r, Q, US, JS, ssum, c0);
        wave_sync();
        const int nq = Q - c0 < CH ? Q - c0 : CH;
#pragma unroll
        for (int s = 0; s < R; ++s)
          if (live[s])
            for (int j = 0; j < nq; ++j)
              gacc[s] = fma(US[j * M + aa[s]], wphiL[(c0 + j) * kp + ii[s]], gacc[s]);
        if (!one_chunk) wave_sync();
      }
      return okp;
    };
    int ok = group_all(grad_pass());

    double g[R];
    auto gradient = [&]() -> double {
      double e2[M];
#pragma unroll
      for (int b = 0; b < M; ++b) e2[b] = 0.0;
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const double gs = live[s] ? gacc[s] - uh[s] : 0.0;
        g[s] = gs;
#pragma unroll
        for (int b = 0; b < M; ++b) e2[b] += (aa[s] == b) ? gs * gs : 0.0;
      }
      // sum over variables of the Euclidean norm over modes (eq:tauCrit)
      double res = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) res += sqrt(group_sum<G>(e2[b]));
      return res;
    };

    double res = 0.0;
#pragma unroll
    for (int s = 0; s < R; ++s) g[s] = 0.0;
    if (ok) res = gradient();
    else status |= kStRealizability;

    constexpr bool reuse = (PREC & 2) != 0;  // inexact-Hessian variant
    bool chord = true;
    // the cell's stored inverse is valid: read once, then kept in step with
    // the flag this cell writes (no re-read of its own write)
    bool have_inv = false;
    if constexpr (reuse) have_inv = P.hinv_ok[cell] == 1;  // 2: handed on without one
    float* Hc = nullptr;  // the cell's stored block of -H^-1, [nc][nc] by column
    if constexpr (reuse)
      Hc = P.hinv + static_cast<size_t>(P.hinv_slot ? P.hinv_slot[cell] : cell) * P.hinv_stride;

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
      // ---- inexact-Hessian Newton: a step from the stored inverse while
      // such steps contract, else a fresh Hessian (inverted and stored)
      double row[R][NP];
      double d[R];
      bool fresh = true;
      if constexpr (reuse) {
        if (chord && have_inv) {  // uniform in the group
          fresh = false;
          // only the cell's n x n block is stored; the mat-vec below reads
          // live rows only, and their entries beyond column n are zero
#pragma unroll
          for (int s = 0; s < R; ++s)
#pragma unroll
            for (int c = 0; c < NP; ++c)
              row[s][c] = (live[s] && c < nc) ? static_cast<double>(Hc[c * nc + ro[s]]) : 0.0;
        }
      }
      if (fresh) {
        // ---- Hessian rows in registers; identity beyond the nc unknowns
#pragma unroll
        for (int s = 0; s < R; ++s)
#pragma unroll
          for (int c = 0; c < NP; ++c) row[s][c] = 0.0;
        {
          int aidx[R][M];
          double live_f[R];
#pragma unroll
          for (int s = 0; s < R; ++s) {
            live_f[s] = live[s] ? 1.0 : 0.0;
#pragma unroll
            for (int b = 0; b < M; ++b) aidx[s][b] = Packed<M>::idx(aa[s], b);
          }
          // the nodes in the same ascending order; with several chunks the
          // ansatz of each chunk is evaluated again for the current dual
          auto node_term = [&](const int q, const double* Jq) {
            double sb[R][M];
#pragma unroll
            for (int s = 0; s < R; ++s) {
              const double wi = wphiL[q * kp + ii[s]] * live_f[s];
#pragma unroll
              for (int b = 0; b < M; ++b) sb[s][b] = Jq[aidx[s][b]] * wi;
            }
            const_dptr ph = phiC + q * kg;  // uniform: scalar loads
#pragma unroll
            for (int c = 0; c < NP; ++c) {
              const double v = ph[c / M];
#pragma unroll
              for (int s = 0; s < R; ++s) row[s][c] = fma(sb[s][c % M], v, row[s][c]);
            }
          };
          if (one_chunk) {
            for (int q = 0; q < Q; ++q) node_term(q, JS + q * NJ);
          } else {
            for (int c0 = 0; c0 < Q; c0 += CH) {
              double sdum = 0.0;
              (void)eval_nodes<M>(P, lamS, Nc, phiL, wphiL, kp, c0 + r, Q, US, JS, sdum, c0);
              wave_sync();
              const int nq = Q - c0 < CH ? Q - c0 : CH;
              for (int j = 0; j < nq; ++j) node_term(c0 + j, JS + j * NJ);
              wave_sync();
            }
          }
#pragma unroll
          for (int s = 0; s < R; ++s)
#pragma unroll
            for (int c = 0; c < NP; ++c)
              row[s][c] = (live[s] && c < nc) ? row[s][c] : (c == ro[s] ? 1.0 : 0.0);
        }

        if constexpr (reuse) {
          // ---- in-place symmetric sweep: H <- -H^-1 (SPD, no pivoting).
          // Step k: pivot p = h_kk; h_kk <- -1/p; row and column k divided by
          // p; h_ij -= h_ik h_kj / p elsewhere.  The matrix stays symmetric,
          // so the pivot row is the broadcast pivot column for every lane; the
          // pivot lane scales its row by 1/p with the multiplier 1/p - 1
          // against that column.
          int pd_ok = 1;
          if constexpr (kDpp) {
            auto halves = [&](double v, double& lo, double& hi) __attribute__((always_inline)) {
              if constexpr (G == 32) {
                group32_halves(v, lo, hi);
              } else {
                lo = v;
                hi = v;
              }
            };
            static_for<0, NP>([&](auto kc) __attribute__((always_inline)) {
              constexpr int k = decltype(kc)::value;
              if (k < kmax) {
                double clo, chi;
                halves(row[0][k], clo, chi);
                const double piv = (k < 16) ? row_bcast<k % 16>(clo) : row_bcast<k % 16>(chi);
                pd_ok &= piv > 0.0 ? 1 : 0;
                const double rp = recip(piv);
                const double f = row[0][k] * rp;
                const double mul = (r == k) ? rp - 1.0 : -f;
                dpp_guard(clo, chi);
                static_for<0, NP>([&](auto jc) __attribute__((always_inline)) {
                  constexpr int j = decltype(jc)::value;
                  if constexpr (j == 16) dpp_guard(clo, chi);
                  if constexpr (j != k)
                    fmac_row_bcast<j % 16>(row[0][j], (j < 16) ? clo : chi, mul);
                });
                row[0][k] = (r == k) ? -rp : f;
              }
              __builtin_amdgcn_sched_barrier(0);
            });
          } else {
#pragma unroll
            for (int s = 0; s < R; ++s) cA[ro[s]] = row[s][0];
            wave_sync();
            // compile-time steps and columns: every register index static
            static_for<0, NP>([&](auto kc) __attribute__((always_inline)) {
              constexpr int k = decltype(kc)::value;
              if (k < nc) {
                const double* A = cA + (k & 1) * NP;
                double* An = cA + ((k + 1) & 1) * NP;
                const double piv = A[k];
                pd_ok &= piv > 0.0 ? 1 : 0;
                const double rp = recip(piv);
                double f[R], mul[R];
#pragma unroll
                for (int s = 0; s < R; ++s) {
                  f[s] = row[s][k] * rp;
                  mul[s] = (ro[s] == k) ? rp - 1.0 : -f[s];
                }
                if constexpr (k + 1 < NP) {  // publish the next column first
                  const double c1 = A[k + 1];
#pragma unroll
                  for (int s = 0; s < R; ++s) {
                    row[s][k + 1] = fma(mul[s], c1, row[s][k + 1]);
                    An[ro[s]] = row[s][k + 1];
                  }
                }
                // the column read entry by entry (a whole column in registers
                // beside the whole row would spill)
                static_for<0, NP>([&](auto jc) __attribute__((always_inline)) {
                  constexpr int j = decltype(jc)::value;
                  if constexpr (j != k && j != k + 1) {
                    const double cj = A[j];
#pragma unroll
                    for (int s = 0; s < R; ++s) row[s][j] = fma(mul[s], cj, row[s][j]);
                  }
                });
#pragma unroll
                for (int s = 0; s < R; ++s) row[s][k] = (ro[s] == k) ? -rp : f[s];
                wave_sync();
              }
            });
          }
          if (!group_all(pd_ok)) {
            status |= kStPivot;
            break;
          }
#pragma unroll
          for (int s = 0; s < R; ++s)
#pragma unroll
            for (int c = 0; c < NP; ++c)
              if (live[s] && c < nc) Hc[c * nc + ro[s]] = static_cast<float>(row[s][c]);
          if (r == 0) P.hinv_ok[cell] = 1;
          have_inv = true;
        } else {
          // ---- Gauss-Jordan solve H d = g without pivoting (H is SPD).  In the
          // symmetric Schur complement the pivot row equals the pivot column, so
          // a broadcast of the column serves all rows and the eliminated system
          // needs no back-substitution.
          double x[R];
          int pd_ok = 1;
          if constexpr (kDpp) {
            // column entry j lives in lane j of the group; lanes 16..31 of a
            // 32-lane group are reached through the swapped copy
            auto halves = [&](double v, double& lo, double& hi) __attribute__((always_inline)) {
              if constexpr (G == 32) {
                group32_halves(v, lo, hi);
              } else {
                lo = v;
                hi = v;
              }
            };
            double dg = 1.0, xv = g[0];
            static_for<0, NP>([&](auto kc) __attribute__((always_inline)) {
              constexpr int k = decltype(kc)::value;
              if (k < kmax) {
                double clo, chi, xlo, xhi;
                halves(row[0][k], clo, chi);
                halves(xv, xlo, xhi);
                const double piv = (k < 16) ? row_bcast<k % 16>(clo) : row_bcast<k % 16>(chi);
                const double gk = (k < 16) ? row_bcast<k % 16>(xlo) : row_bcast<k % 16>(xhi);
                pd_ok &= piv > 0.0 ? 1 : 0;
                if (r == k) dg = piv;
                const double f = (r == k) ? 0.0 : row[0][k] * recip1(piv);
                const double negf = -f;
                xv = fma(-f, gk, xv);
                dpp_guard(clo, chi);
                static_for<k + 1, NP>([&](auto jc) __attribute__((always_inline)) {
                  constexpr int j = decltype(jc)::value;
                  if constexpr (j == 16 && k + 1 < 16) dpp_guard(clo, chi);
                  fmac_row_bcast<j % 16>(row[0][j], (j < 16) ? clo : chi, negf);
                });
              }
              // one step at a time: interleaving steps keeps every step's
              // multipliers and broadcasts live at once
              __builtin_amdgcn_sched_barrier(0);
            });
            if (!group_all(pd_ok)) {
              status |= kStPivot;
              break;
            }
            x[0] = xv;
            d[0] = live[0] ? xv * recip(dg) : 0.0;
          } else {
            // LDS broadcast: the step reads the whole column in one batch,
            // updates and publishes the next column first, then the rest of the
            // row while that write lands
#pragma unroll
            for (int s = 0; s < R; ++s) {
              x[s] = g[s];
              cA[ro[s]] = row[s][0];
            }
            if (r == 0) cX[0] = x[0];
            wave_sync();
#pragma unroll
            for (int k = 0; k < NP; ++k) {
              // steps beyond the cell's unknowns would only touch the identity block
              if (k < nc) {
                const double* A = cA + (k & 1) * NP;
                double* An = cA + ((k + 1) & 1) * NP;
                double col[NP];
#pragma unroll
                for (int j = k; j < NP; ++j) col[j] = A[j];
                const double gk = cX[k & 1];
                const double piv = col[k];
                pd_ok &= piv > 0.0 ? 1 : 0;
                if (r == k % G) cP[k] = piv;
                const double rp = recip(piv);
                double f[R];
#pragma unroll
                for (int s = 0; s < R; ++s) {
                  f[s] = (ro[s] == k) ? 0.0 : row[s][k] * rp;
                  x[s] = fma(-f[s], gk, x[s]);
                }
                if (k + 1 < NP) {
#pragma unroll
                  for (int s = 0; s < R; ++s) {
                    row[s][k + 1] = fma(-f[s], col[k + 1], row[s][k + 1]);
                    An[ro[s]] = row[s][k + 1];
                  }
                  if (r == (k + 1) % G) cX[(k + 1) & 1] = x[(k + 1) / G];
                }
#pragma unroll
                for (int j = k + 2; j < NP; ++j)
#pragma unroll
                  for (int s = 0; s < R; ++s) row[s][j] = fma(-f[s], col[j], row[s][j]);
                wave_sync();
              }
            }
            if (!group_all(pd_ok)) {
              status |= kStPivot;
              break;
            }
            wave_sync();
#pragma unroll
            for (int s = 0; s < R; ++s) d[s] = live[s] ? x[s] * recip(cP[ro[s]]) : 0.0;
          }

        }  // exact solve
      }  // fresh Hessian
      if constexpr (reuse) {
        // d = H^-1 g = -(rows of -H^-1) g, g through the group's LDS area
        // (free until the line search writes the trial dual)
#pragma unroll
        for (int s = 0; s < R; ++s) lamS[ro[s]] = g[s];
        wave_sync();
#pragma unroll
        for (int s = 0; s < R; ++s) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < NP; ++j) acc = fma(row[s][j], lamS[j], acc);
          d[s] = live[s] ? -acc : 0.0;
        }
        wave_sync();
      }
      // ---- step length
      const bool ls = !P.one_shot && res > 1e-6;
      double L0 = 0.0, slope = 0.0;
      if (ls) {
        double l0 = ssum, sl = 0.0;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          l0 -= lam[s] * uh[s];
          sl += g[s] * d[s];
        }
        L0 = group_sum<G>(l0);
        slope = group_sum<G>(sl);
      }
      double t = 1.0, lt[R];
#pragma unroll
      for (int s = 0; s < R; ++s) lt[s] = lam[s];
      int accepted = 0;
#pragma unroll 1
      for (int h = 0; h <= 60; ++h) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
          lt[s] = lam[s] - t * d[s];
          lamS[ro[s]] = lt[s];
        }
        wave_sync();
        ok = group_all(grad_pass());
        if (!ls) {
          accepted = 1;
          break;
        }
        if (ok) {
          double lt_sum = ssum;
#pragma unroll
          for (int s = 0; s < R; ++s) lt_sum -= lt[s] * uh[s];
          const double Lt = group_sum<G>(lt_sum);
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
#pragma unroll
      for (int s = 0; s < R; ++s) lam[s] = lt[s];
      ++its;
      nfresh += fresh ? 1 : 0;
      if (!ok) {
        status |= kStRealizability;
        break;
      }
      const double res_old = res;
      res = gradient();
      // a step from the stored inverse must contract the residual by
      // theta, else the inverse is retired: the cell's next iteration, in this or a
      // later step (one-shot: the next pseudo-time step), assembles afresh
      if (!fresh && !(res <= P.reuse_theta * res_old)) {
        chord = false;
        if (r == 0) P.hinv_ok[cell] = 0;
        have_inv = false;
      }
      if (P.one_shot) break;
    }

    // ---- write back: dual, nodal ansatz, wave speeds
#pragma unroll
    for (int s = 0; s < R; ++s)
      if (live[s]) P.lam[gidx[s]] = lam[s];
    // (several chunks: the ansatz of the final dual once more, node by node)
    for (int q = r; q < Q; q += G) {
      double u[M];
      if (one_chunk) {
#pragma unroll
        for (int b = 0; b < M; ++b) u[b] = US[q * M + b];
      } else {
        double L[M], J[NJ], ss;
#pragma unroll
        for (int a = 0; a < M; ++a) L[a] = 0.0;
        const double* ph = phiL + q * kp;
        for (int i = 0; i < Nc; ++i)
#pragma unroll
          for (int a = 0; a < M; ++a) L[a] = fma(lamS[i * M + a], ph[i], L[a]);
        (void)closure<M>(P.cp, L, u, J, ss);
      }
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
    // iterations, fresh ones and the listed flag packed exactly in one double
    // (its <= max_newton < 1024)
    stats[(wave * CPW + grp) * 2 + 0] =
        static_cast<double>(its + 1024 * nfresh + (cell >= 0 ? 1048576 : 0));
    stats[(wave * CPW + grp) * 2 + 1] = static_cast<double>(status);
  }
  if (lane == 0) {
    stats[2 * waves * CPW + 2 * wave] = sx;
    stats[2 * waves * CPW + 2 * wave + 1] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum_its = 0, max_its = 0, listed = 0, sum_fresh = 0;
    unsigned st = 0;
    double mx = 0.0, my = 0.0;
    for (int k = 0; k < waves * CPW; ++k) {
      const unsigned long long v = static_cast<unsigned long long>(stats[2 * k]);
      const unsigned long long it = v & 1023ull;
      sum_its += it;
      max_its = it > max_its ? it : max_its;
      sum_fresh += (v >> 10) & 1023ull;
      listed += v >> 20;
      st |= static_cast<unsigned>(stats[2 * k + 1]);
    }
    for (int w = 0; w < waves; ++w) {
      mx = nan_max(mx, stats[2 * waves * CPW + 2 * w]);
      my = nan_max(my, stats[2 * waves * CPW + 2 * w + 1]);
    }
    const int slot = (blk & (kSlots - 1)) * kSlotStride;
    if (P.mode == 0) {
      unsigned long long* bs = P.blk_stats + kBlkStats * static_cast<size_t>(blk);
      bs[0] += sum_its;
      if (max_its > bs[1]) bs[1] = max_its;
      bs[2] += listed;
      bs[3] += sum_fresh;
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

// The inexact-Hessian variant keeps the whole inverse row live through the
// sweep; for NP <= 32 it is held to the exact kernel's two wavefronts per SIMD.
template <int M, int NP, int PREC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(((PREC & 3) == 2 && NP <= 32) ? 2 : 1)))
void newton_kernel(DualParams P) {
  if (P.pend) {  // the handed-on cells, block by block
    const int cpb = (blockDim.x >> 6) * NewtonCfg<M, NP>::CPW;
    const int n = static_cast<int>(P.ctrl->pend_len[P.parity][P.cls]);
    for (int vb = blockIdx.x; vb * cpb < n; vb += gridDim.x) {
      newton_body<M, NP, PREC>(P, vb);
      __syncthreads();
    }
    return;
  }
  newton_body<M, NP, PREC>(P, blockIdx.x);
}

// Problem k of a batched launch owns blocks begin[k] .. begin[k+1]-1.
__device__ __forceinline__ int batch_problem(const int* __restrict__ begin, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#ifdef IPM_HOST_UNIT  // defined once, in the host runtime's unit that launches it
// Block offsets of a batched list-mode Newton launch, from the lists the
// flux update filled: problem k gets ceil(listed_k / per_block) blocks from
// begin[k] on, so all listed cells sit in the first blocks of the grid.  It
// also clears each problem's next-step lists and speed slots (the duty of
// the problem's first Newton launch of the step, flagged reset_next).  One
// wavefront; lane j takes problem k0 + j of each group of 64 (its flags and
// list lengths are independent loads), the block counts are scanned across
// the lanes, and the resets run problem by problem on all lanes.
__global__ __launch_bounds__(64) void batch_prefix_kernel(const DualParams* __restrict__ PP, int n,
                                                          int per_block, int* __restrict__ begin) {
  const int lane = threadIdx.x;
  int acc = 0;
  if (lane == 0) begin[0] = 0;
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int k = k0 + lane;
    int blocks = 0, reset = 0, parity = 0;
    StepCtrl* C = nullptr;
    if (k < n) {
      const DualParams& P = PP[k];
      C = P.ctrl;
      parity = P.parity;
      if (!(C->done[parity] || C->status)) {
        const unsigned* len = C->list_len + list_len_index(parity, P.cls, 0);
        int listed = 0;
        for (int s = 0; s < kSlots; ++s) listed += min(static_cast<int>(len[s * kSlotStride]), P.list_cap);
        blocks = (listed + per_block - 1) / per_block;
        reset = P.reset_next;
      }
    }
    int v = blocks;  // inclusive scan over the group's problems
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (k < n) begin[k + 1] = acc + v;
    acc += __shfl(v, 63, 64);
    unsigned long long todo = __ballot(reset != 0);
    while (todo != 0ull) {
      const int j = __ffsll(static_cast<long long>(todo)) - 1;
      todo &= todo - 1ull;
      StepCtrl* Cj = reinterpret_cast<StepCtrl*>(
          __shfl(static_cast<long long>(reinterpret_cast<uintptr_t>(C)), j, 64));
      reset_next_ctrl(Cj, __shfl(parity, j, 64));
    }
  }
}
#endif

template <int M, int NP, int PREC = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(((PREC & 3) == 2 && NP <= 32) ? 2 : 1)))
void newton_batched(const DualParams* __restrict__ PP, const int* __restrict__ begin, int n) {
  const int k = batch_problem(begin, n, blockIdx.x);
  if (PP[k].pend) {
    const DualParams& P = PP[k];
    const int cpb = (blockDim.x >> 6) * NewtonCfg<M, NP>::CPW;
    const int n = static_cast<int>(P.ctrl->pend_len[P.parity][P.cls]);
    for (int vb = blockIdx.x - begin[k]; vb * cpb < n; vb += kPendBlocks) {
      newton_body<M, NP, PREC>(P, vb);
      __syncthreads();
    }
    return;
  }
  newton_body<M, NP, PREC>(PP[k], blockIdx.x - begin[k]);
}

}  // namespace ipm
