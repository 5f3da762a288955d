// libipm: C ABI, problem state on the device, kernel dispatch.
//
// The host validates problems, builds the quadrature and basis tables once
// per problem, and enqueues kernels; every step of the method (IC
// projection, dual solves, flux quadrature, moment update, time step,
// residual) runs on the GPU.  See include/ipm.h for the ABI contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ipm.h"
// this unit defines the non-template kernels it launches itself
#define IPM_HOST_UNIT
#include "chord.hpp"
#include "chord_big.hpp"
#include "dual_big.hpp"
#include "kernel_select.hpp"
#include "tables.hpp"

using namespace ipm;

namespace {

thread_local std::string g_create_error;

// Newton launch configuration of one size class of a problem's cells
struct DualClass {
  bool configured = false;  // kernel chosen (cells of the class, or the ghosts' full size)
  int prec = 0;             // 1: BF16-split MFMA Hessian (precision form, workgroup kernel)
  int bcache = 1;           // precision form: B fragments cached in LDS (when they fit)
  int NP = 8;               // lanes per cell (small kernel) or 16 T (workgroup kernel)
  int T = 0;                // > 0: workgroup kernel with T x T tiles
  int waves = 4;            // small kernel: wavefronts per block
  size_t lds = 0;
  int count = 0;            // cells the class plans for (all cells when levels adapt)
  int order_len = 0;        // cells of the class at set-up (length of d_order)
  int cap = 0;              // list capacity per slot
  int* d_lists = nullptr;   // [2][64][cap] Newton lists by step parity
  int* d_order = nullptr;   // [count] cells of the class ascending (null: all cells)
  int blk_off = 0, blk_cnt = 0;  // range in the block-statistics array
  bool merged = false;      // its cells go to the lists of a larger class
  float* d_hinv = nullptr;  // inexact-Hessian Newton: stored inverses of the class's cells (FP32)
  int n_min = 0, n_max = 0; // unknowns of the cells its launches solve (set-up)
  // register-row inexact-Hessian classes: chord steps in a kernel of their
  // own, then the full kernel over the cells it handed on
  bool chord = false;
  int chord_kl = 1;         // table columns the chord kernel stages (its cells' modes)
  int chord_waves = 4;
  size_t chord_lds = 0;
  int cblk_off = 0, cblk_cnt = 0;  // the chord kernel's block statistics
  int* d_pend = nullptr;            // [count] cells the chord kernel hands on
};

// Problems up to this many cells are latency bound: one Newton launch for
// two adjacent small-cell classes beats one launch each.
constexpr int kMergeCells = 32768;

struct Problem {
  int eq = 0, M = 1, dim = 1, p = 1, degree = 0, N = 1, Q = 1, kp = 1, UG = 16;
  int cls_modes[kCls] = {};  // most modes of a cell in each size class (before merging)
  int full_cls = 0;  // class of a cell with all N modes (ghosts)
  DualClass cls[kCls];
  int nx = 1, ny = 1, cells = 1;
  int flux = 0, max_newton = 100, one_shot = 0, precision = 0;
  int bc[4] = {0, 0, 0, 0};
  double cfl = 0.5, t_end = 0.0, tau = 1e-10, steady_eps = 0.0;
  double dx = 1.0, dy = 1.0, vol = 1.0;
  ClosureParams cp{};
  bool uneven = false;
  // dynamic adaptivity: levels move between min_degree and degree
  int adapt = 0, min_degree = 1;
  double delta_lo = 0.0, delta_hi = 0.0;
  Retard* d_retard = nullptr;  // refinement retardation state (null: none)
  unsigned cls_map = 0x76543210u;  // 4 bits per size class: the class whose lists take its cells
  // Newton launches run over the step's work lists (else over all cells of
  // each class in a fixed order: one-shot with fixed degrees)
  bool lists() const { return !one_shot || adapt; }
  double* d_phi = nullptr;
  double* d_wphi = nullptr;
  double* d_u[2] = {nullptr, nullptr};
  double* d_lam = nullptr;
  double* d_nodal = nullptr;
  double* d_ghost = nullptr;
  double* d_res = nullptr;
  // chord kernels on the Euler entropy: the update leaves each cell's
  // warm-start dual gradient (in the old moments' buffer) and <s_*> [cells]
  bool gwarm = false;
  double* d_s0 = nullptr;
  bool upd_stage = false;  // the update stages its basis table in LDS
  unsigned long long* d_blk = nullptr;
  // modes per cell read by the steps of each parity (one buffer when fixed;
  // adaptive: the update of a step writes the other parity's buffer)
  int8_t* d_cellN[2] = {nullptr, nullptr};
  double* d_ctp = nullptr;  // analytic SG flux: triple products [N][N][N]
  // inexact-Hessian Newton: 1 = cells on the workgroup kernel, 2 = every cell
  int hessian_reuse = 0;
  double reuse_theta = 0.5;
  unsigned char* d_hinv_ok = nullptr;  // [cells] stored inverse valid
  int* d_hinv_slot = nullptr;          // [cells] slot within the class's inverses
  // with adaptive levels: one slot per cell of the largest class's size (a
  // cell moves between classes; a level change retires its inverse)
  float* d_hinv_all = nullptr;
  long long hinv_all_stride = 0;
  // the class's inverses and their size (set per launch)
  void set_hinv(DualParams& d, const DualClass& D) const {
    d.hinv = hinv_all_stride ? d_hinv_all : D.d_hinv;
    d.hinv_ok = d_hinv_ok;
    d.hinv_stride = hinv_all_stride ? hinv_all_stride : static_cast<long long>(D.NP) * D.NP;
    d.hinv_slot = hinv_all_stride ? nullptr : d_hinv_slot;
    d.reuse_theta = reuse_theta;
  }
  StepCtrl* d_ctrl = nullptr;
  long long step_index = 0;
  size_t bytes = 0;    // device bytes allocated
  size_t charged = 0;  // bytes charged against the context's budget
  int upd_blocks = 1, dual_blocks = 1;
  size_t upd_lds = 0;
  int upd_waves = 4;  // wavefronts per update block (fewer when the node tiles fill LDS)
};

// One launch of a batched step: a Newton launch of one kernel template over
// several problems' size classes, an update launch over several problems, or
// a single problem's steady-residual kernel.
struct BatchLaunch {
  int kind = 0;  // 0: Newton (batched), 1: update (batched), 2: residual
  bool lists = false;  // Newton over the step's lists: block offsets computed on the device
  int per_block = 1;   // cells per Newton block
  const void* fn = nullptr;
  int blocks = 0, threads = 0;
  size_t lds = 0;
  size_t pofs = 0;  // first entry in the phase's params array of this kind
  int bofs = 0;     // first entry in the begin array
  int n = 0;        // problems (entries) in the launch
  int pid = -1;     // residual: problem id
  int parity = 0;   // residual: step parity
  int M = 0, lanes = 0, workgroup = 0, variant = 0;  // Newton: kernel shape (timing records)
  int stage = 1;  // Newton: 0 chord kernels, 1 the others (after stage 0)
};

// Problems stepped together: both step parities prepared once, as launch
// lists and as instantiated graphs.
struct BatchPlan {
  std::vector<int> ids;
  std::vector<long long> step0;  // step_index of each problem when built
  long long steps_done = 0;
  unsigned long long gen = 0;    // context generation when built
  std::vector<BatchLaunch> launches[2];
  DualParams* d_dp = nullptr;    // [2][nd]
  UpdateParams* d_up = nullptr;  // [2][nu]
  int* d_begin = nullptr;
  int* d_dev_begin = nullptr;  // device-computed block offsets of list-mode Newton launches
  size_t nd = 0, nu = 0;
  size_t cap_dp = 0, cap_up = 0, cap_begin = 0;  // element capacities of the owned arrays
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  bool owned = true;  // false: the arrays live in the static scratch (not freed)
  unsigned long long scratch_tag = 0;  // static plans: upload this plan's contents carry
  ~BatchPlan() {
    for (int k = 0; k < 2; ++k) {
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
    }
    if (!owned) return;
    if (d_dp) (void)hipFree(d_dp);
    if (d_up) (void)hipFree(d_up);
    if (d_begin) (void)hipFree(d_begin);
    if (d_dev_begin) (void)hipFree(d_dev_begin);
  }
};

// Device scratch of ipm_step_static: the batched launches' parameter arrays
// and block offsets, for callers that cannot allocate.  One copy per GPU,
// held until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// name is a host-side stand-in, not a device address).
constexpr size_t kStaticScratchBytes = 512 * 1024;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Per device: the scratch's device address and which upload it holds.
struct ScratchSlot {
  unsigned char* ptr = nullptr;
  const void* owner = nullptr;   // context whose plan the scratch holds
  unsigned long long tag = 0;    // that upload
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;
unsigned long long g_scratch_uploads = 0;

}  // namespace

struct ipm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, used = 0;
  int max_problems = 1024;
  std::vector<std::unique_ptr<Problem>> problems;
  std::string err;
  size_t max_lds = 64 * 1024;  // dynamic LDS bytes one block may use
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pairs: dual start/stop, update start/stop
  size_t ev_used = 0;
  // per batched Newton launch while timing: its shape key and event pair
  struct LaunchRec {
    int M, lanes, workgroup, variant, threads;
    size_t ev;  // index of the start event in lev
  };
  std::vector<LaunchRec> lrec;
  std::vector<hipEvent_t> lev;
  size_t lev_used = 0;
  std::vector<ipm_launch_time> ltimes;  // totals of the last timing window
  unsigned long long gen = 0;              // bumped when problems or launch shapes change
  std::unique_ptr<BatchPlan> batch;        // cached plan of the last batched ipm_step
  // serving loop's poll: the control-block heads of the active problems
  // gathered on the device, one copy into pinned host memory per round
  unsigned long long* d_poll = nullptr;
  unsigned long long* h_poll = nullptr;
  size_t poll_cap = 0;  // problems
  std::map<std::string, int> tuned_waves;  // autotuner: wavefronts per Newton block by shape
  // ipm_step_static: this device's scratch address, the plan it stepped last
  // and the host copies of that plan's arrays
  unsigned char* scratch = nullptr;
  std::unique_ptr<BatchPlan> static_plan;
  std::vector<DualParams> static_dps;
  std::vector<UpdateParams> static_ups;
  std::vector<int> static_begins;
};

namespace {

ipm_status fail(ipm_ctx* ctx, ipm_status st, const std::string& msg) {
  if (ctx)
    ctx->err = msg;
  else
    g_create_error = msg;
  return st;
}

#define HIPCHK(ctx, expr)                                                            \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(ctx, IPM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int components(int eq) { return eq == IPM_BURGERS_1D ? 1 : (eq == IPM_EULER_1D ? 3 : 4); }

int pow2_at_least(int n, int lo) {
  int v = lo;
  while (v < n) v <<= 1;
  return v;
}

DualFn pick_big(int M, int T, int prec = 0) {
  if (M == 1) return big_pick<1>(T, prec);
  if (M == 4) return big_pick<4>(T, prec);
  return nullptr;
}

// LDS of a workgroup-kernel variant (the reuse bit's matrix-vector area is
// added by plan when the variant has no MFMA block area to hold it)
size_t big_lds_bytes(int M, int T, int Q, int kp, int prec = 0, bool bcache = true) {
  auto f = [&](auto tag) -> size_t {
    constexpr int MM = decltype(tag)::value;
    auto g = [&](auto ptag) -> size_t {
      constexpr int PR = decltype(ptag)::value;
      switch (T) {
        case 1: return BigCfg<MM, 1, PR>::lds_bytes(Q, kp, bcache);
        case 2: return BigCfg<MM, 2, PR>::lds_bytes(Q, kp, bcache);
        case 4: return BigCfg<MM, 4, PR>::lds_bytes(Q, kp, bcache);
        case 5: return BigCfg<MM, 5, PR>::lds_bytes(Q, kp, bcache);
        case 6: return BigCfg<MM, 6, PR>::lds_bytes(Q, kp, bcache);
        case 8: return BigCfg<MM, 8, PR>::lds_bytes(Q, kp, bcache);
        default: return BigCfg<MM, 9, PR>::lds_bytes(Q, kp, bcache);
      }
    };
    switch (prec & 3) {
      case 1: return g(std::integral_constant<int, 1>{});
      case 2: return g(std::integral_constant<int, 2>{});
      case 3: return g(std::integral_constant<int, 3>{});
      default: return g(std::integral_constant<int, 0>{});
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  return f(std::integral_constant<int, 4>{});
}

// Register-row kernel variant of a class: exact (0) and inexact-Hessian (2)
// Newton take their single-chunk form (+4) when the cell's lanes hold every
// node at once
int reg_variant(int prec, int T, int NP, int Q) {
  return (T == 0 && (prec == 0 || prec == 2) && Q <= NP) ? (prec | 4) : prec;
}

DualFn pick_dual(int M, int NP, int prec = 0) {
  if (M == 1) return dual_pick<1>(NP, prec);
  if (M == 3) return dual_pick<3>(NP, prec);
  if (M == 4) return dual_pick<4>(NP, prec);
  return nullptr;
}

UpdFn pick_update(int M, int G) {
  if (M == 1) return update_pick<1>(G);
  if (M == 3) return update_pick<3>(G);
  if (M == 4) return update_pick<4>(G);
  return nullptr;
}

SetupFn pick_setup(int M) {
  if (M == 1) return setup_pick<1>();
  if (M == 3) return setup_pick<3>();
  return setup_pick<4>();
}

template <int M, int NP>
using NC = NewtonCfg<M, NP>;

// dynamic LDS bytes of the Newton kernel
size_t chord_lds_bytes(int M, int NP, int Q, int kl, int waves) {
  auto f = [&](auto tag) -> size_t {
    constexpr int MM = decltype(tag)::value;
    switch (NP) {
      case 8: return ChordCfg<MM, 8>::lds_bytes(Q, kl, waves);
      case 16: return ChordCfg<MM, 16>::lds_bytes(Q, kl, waves);
      case 32: return ChordCfg<MM, 32>::lds_bytes(Q, kl, waves);
      default: return ChordCfg<MM, 64>::lds_bytes(Q, kl, waves);
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  if (M == 3) return f(std::integral_constant<int, 3>{});
  return f(std::integral_constant<int, 4>{});
}

size_t chord_big_lds_bytes(int M, int T, int Q, int kl, int waves) {
  auto f = [&](auto tag) -> size_t {
    constexpr int MM = decltype(tag)::value;
    switch (T) {
      case 1: return ChordBigCfg<MM, 1>::lds_bytes(Q, kl, waves);
      case 2: return ChordBigCfg<MM, 2>::lds_bytes(Q, kl, waves);
      case 4: return ChordBigCfg<MM, 4>::lds_bytes(Q, kl, waves);
      case 5: return ChordBigCfg<MM, 5>::lds_bytes(Q, kl, waves);
      case 6: return ChordBigCfg<MM, 6>::lds_bytes(Q, kl, waves);
      case 8: return ChordBigCfg<MM, 8>::lds_bytes(Q, kl, waves);
      default: return ChordBigCfg<MM, 9>::lds_bytes(Q, kl, waves);
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  return f(std::integral_constant<int, 4>{});
}

size_t dual_lds_bytes(int M, int NP, int Q, int kp, int waves) {
  auto f = [&](auto tag) -> size_t {
    constexpr int MM = decltype(tag)::value;
    switch (NP) {
      case 8: return NC<MM, 8>::lds_bytes(Q, kp, waves);
      case 16: return NC<MM, 16>::lds_bytes(Q, kp, waves);
      case 32: return NC<MM, 32>::lds_bytes(Q, kp, waves);
      default: return NC<MM, 64>::lds_bytes(Q, kp, waves);
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  if (M == 3) return f(std::integral_constant<int, 3>{});
  return f(std::integral_constant<int, 4>{});
}

// cells one wavefront of the Newton kernel works on
int dual_cells_per_wave(int M, int NP) {
  auto f = [&](auto tag) -> int {
    constexpr int MM = decltype(tag)::value;
    switch (NP) {
      case 8: return NC<MM, 8>::CPW;
      case 16: return NC<MM, 16>::CPW;
      case 32: return NC<MM, 32>::CPW;
      default: return NC<MM, 64>::CPW;
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  if (M == 3) return f(std::integral_constant<int, 3>{});
  return f(std::integral_constant<int, 4>{});
}

// basis-table columns the Newton kernel's Hessian segments read
int dual_table_columns(int M, int NP) {
  auto f = [&](auto tag) -> int {
    constexpr int MM = decltype(tag)::value;
    switch (NP) {
      case 8: return NC<MM, 8>::KCOL;
      case 16: return NC<MM, 16>::KCOL;
      case 32: return NC<MM, 32>::KCOL;
      default: return NC<MM, 64>::KCOL;
    }
  };
  if (M == 1) return f(std::integral_constant<int, 1>{});
  if (M == 3) return f(std::integral_constant<int, 3>{});
  return f(std::integral_constant<int, 4>{});
}

Problem* get(ipm_ctx* ctx, int id) {
  if (!ctx || id < 0 || id >= static_cast<int>(ctx->problems.size())) return nullptr;
  return ctx->problems[id].get();
}

void free_problem(Problem* P) {
  if (!P) return;
  void* ptrs[] = {P->d_phi,   P->d_wphi, P->d_u[0], P->d_u[1],  P->d_lam, P->d_nodal,
                  P->d_ghost, P->d_res,  P->d_blk,  P->d_cellN[0], P->d_ctrl, P->d_retard, P->d_ctp, P->d_hinv_ok, P->d_hinv_slot, P->d_hinv_all,
                  P->d_s0};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (P->d_cellN[1] && P->d_cellN[1] != P->d_cellN[0]) (void)hipFree(P->d_cellN[1]);
  for (DualClass& c : P->cls) {
    if (c.d_lists) (void)hipFree(c.d_lists);
    if (c.d_order) (void)hipFree(c.d_order);
    if (c.d_hinv) (void)hipFree(c.d_hinv);
    if (c.d_pend) (void)hipFree(c.d_pend);
  }
}

// Phi columns a class's Newton kernel stages in LDS: those its rows read
// (the lane groups' padded rows for register rows; 16 T / m for the tiles),
// at most the global table's.  Register rows read a node's row per lane, so
// their stride is made odd (conflict-free banks; the kernel zero-fills a
// column beyond the global table).
int class_kl(int M, int kp, int NP, int T) {
  if (T > 0) return std::min(kp, (16 * T + M - 1) / M);
  return std::min(kp, dual_table_columns(M, NP)) | 1;
}

// shape key of a small-kernel class for the autotuner
std::string tune_key(const Problem& P, const DualClass& D) {
  return std::to_string(P.M) + "," + std::to_string(D.NP) + "," + std::to_string(P.Q) + "," +
         std::to_string(P.kp);
}

// Launch geometry of a problem's kernels.  counts[c]: cells per size class.
ipm_status plan(ipm_ctx* ctx, Problem& P, const int* counts) {
  const int n = P.M * P.N;
  P.full_cls = size_class(n);
  for (int c = 0; c < kCls; ++c) {
    P.cls[c] = DualClass{};
    P.cls[c].count = counts[c];
    P.cls[c].configured = counts[c] > 0 || c == P.full_cls;
  }
  P.kp = P.N;
  for (int c = 0; c < kCls; ++c) {
    DualClass& D = P.cls[c];
    if (!D.configured) continue;
    if (c >= 4) {
      // workgroup per cell; the tile layout needs m | 16 (m = 1 or 4)
      if (16 % P.M != 0)
        return fail(ctx, IPM_E_ARG,
                    "m*N = " + std::to_string(n) + " > 64 unknowns per cell is supported for m = 1 "
                    "and m = 4 only");
      if (n > 144)
        return fail(ctx, IPM_E_ARG, "m*N = " + std::to_string(n) + " unknowns per cell exceeds 144");
      D.T = class_tiles(c);
      D.NP = 16 * D.T;
      // BF16 Hessian up to 96 unknowns: above, its FP32 block area (92 KB
      // at 140 unknowns and 125 nodes) costs more occupancy than the MFMA
      // saves (measured 0.76x the FP64 assembly there)
      D.prec = (P.precision == IPM_PREC_BF16 && D.T <= 6 ? 1 : 0) | (P.hessian_reuse ? 2 : 0);
    } else {
      D.NP = 8 << c;
      // no BF16 Hessian below 65 unknowns; inexact-Hessian Newton on the
      // register-row kernels only when asked for (hessian_reuse = 2)
      D.prec = P.hessian_reuse == 2 ? 2 : 0;
      P.kp = std::max(P.kp, dual_table_columns(P.M, D.NP));
    }
  }
  P.UG = pow2_at_least(std::min(64, std::max(P.Q, n)), 16);
  // update blocks of 4 wavefronts, or fewer when the per-cell node tiles of
  // many quadrature nodes would not fit LDS
  // the weighted basis table goes to LDS up to 16 KiB (short latency for the
  // small, latency-bound problems), else it is read from device memory
  P.upd_stage = static_cast<size_t>(P.Q) * P.kp * sizeof(double) <= 16384;
  const size_t tab = P.upd_stage ? static_cast<size_t>(P.Q) * P.kp : 0;
  auto upd_lds_for = [&](int waves) {
    const size_t cpb = static_cast<size_t>(waves) * (64 / P.UG);
    return sizeof(double) * (tab + 2 * cpb * P.Q * P.M + 256 +
                             (P.flux == IPM_FLUX_SG_ANALYTIC ? static_cast<size_t>(P.N) * P.N * P.N : 0));
  };
  P.upd_waves = 4;
  while (P.upd_waves > 1 && upd_lds_for(P.upd_waves) > ctx->max_lds) P.upd_waves >>= 1;
  const int ucpb = P.upd_waves * (64 / P.UG);
  P.upd_blocks = (P.cells + ucpb - 1) / ucpb;
  P.upd_lds = sizeof(double) * (tab + 2 * static_cast<size_t>(ucpb) * P.Q * P.M + 256 +
                                (P.flux == IPM_FLUX_SG_ANALYTIC ? static_cast<size_t>(P.N) * P.N * P.N : 0));
  if (P.upd_lds > ctx->max_lds) return fail(ctx, IPM_E_ARG, "quadrature too large for the update kernel");
  P.dual_blocks = 0;
  for (int c = 0; c < kCls; ++c) {
    DualClass& D = P.cls[c];
    if (!D.configured) continue;
    if (D.T == 0) {
      // wavefronts per block: the most wavefronts per CU that LDS allows
      // (160 KiB per CU); ties go to the larger block
      auto per_cu = [&](int w) {
        const size_t b = dual_lds_bytes(P.M, D.NP, P.Q, class_kl(P.M, P.kp, D.NP, 0), w);
        return b > ctx->max_lds ? 0 : w * static_cast<int>(std::min<size_t>(4, (160 * 1024) / b));
      };
      D.waves = 4;
      for (int w : {2, 1})
        if (per_cu(w) > per_cu(D.waves)) D.waves = w;
      auto tw = ctx->tuned_waves.find(tune_key(P, D));
      if (tw != ctx->tuned_waves.end() &&
          dual_lds_bytes(P.M, D.NP, P.Q, class_kl(P.M, P.kp, D.NP, 0), tw->second) <= ctx->max_lds)
        D.waves = tw->second;
      D.lds = dual_lds_bytes(P.M, D.NP, P.Q, class_kl(P.M, P.kp, D.NP, 0), D.waves);
      // many nodes: the per-cell node buffers of a wavefront's cells leave
      // fewer than two wavefronts per CU (or do not fit), so the class runs
      // on the workgroup-per-cell kernel
      if (per_cu(D.waves) < 2 && 16 % P.M == 0) {
        D.T = std::max(1, D.NP / 16);
        D.NP = 16 * D.T;
        D.prec = P.hessian_reuse ? 2 : 0;
      }
    }
    if (D.T > 0) {
      D.waves = 4;
      D.bcache = 1;
      // the inexact-Hessian areas (17 x 16T doubles) live in the MFMA block
      // area when there is one
      const size_t extra = ((D.prec & 2) && !(D.prec & 1)) ? sizeof(double) * 17 * 16 * D.T : 0;
      const int kl = class_kl(P.M, P.kp, D.NP, D.T);
      D.lds = big_lds_bytes(P.M, D.T, P.Q, kl, D.prec, true) + extra;
      if (D.prec & 1) {
        // build the B fragments on the fly instead of caching them when the
        // cache does not fit, or when it would cost the second workgroup
        // per CU that the registers allow (160 KiB of LDS per CU)
        const size_t lean = big_lds_bytes(P.M, D.T, P.Q, kl, D.prec, false) + extra;
        const size_t cu = 160 * 1024;
        if (D.lds > ctx->max_lds || (2 * D.lds > cu && 2 * lean <= cu)) {
          D.bcache = 0;
          D.lds = lean;
        }
      }
    }
    if (D.lds > ctx->max_lds)
      return fail(ctx, IPM_E_ARG, "quadrature too large for the dual kernel's LDS tiles (Q = " +
                                      std::to_string(P.Q) + ")");
  }
  // a small problem's cells of the next smaller small-cell class run in the
  // largest small-cell class's launch (their unknowns fit its lane groups;
  // the kernel handles cells of any size up to its own)
  P.cls_map = 0x76543210u;
  // (not with inexact-Hessian Newton: the stored inverses are per class)
  if (P.lists() && P.cells <= kMergeCells && P.hessian_reuse != 2) {
    int top = -1;
    for (int c = 0; c < 4; ++c)
      if (P.cls[c].configured && P.cls[c].count > 0 && P.cls[c].T == 0) top = c;
    if (top > 0) {
      DualClass& L = P.cls[top - 1];
      if (L.configured && L.count > 0 && L.T == 0) {
        L.merged = true;
        P.cls[top].count = std::min(P.cells, P.cls[top].count + L.count);
        P.cls_map = (P.cls_map & ~(15u << (4 * (top - 1)))) | (static_cast<unsigned>(top) << (4 * (top - 1)));
      }
    }
  }
  for (int c = 0; c < kCls; ++c) {
    DualClass& D = P.cls[c];
    if (!D.configured) continue;
    // list l receives the routed cells of update blocks b = l (mod 64)
    D.cap = (D.count > 0 && !D.merged)
                ? std::min(((P.upd_blocks + kSlots - 1) / kSlots) * ucpb, D.count) : 0;
    // block statistics sized for one wavefront per block, the smallest the
    // autotuner may choose
    const int per_block = D.T > 0 ? 1 : dual_cells_per_wave(P.M, D.NP);
    const int items = std::max(kSlots * D.cap, D.count);
    D.blk_off = P.dual_blocks;
    D.blk_cnt = (items + per_block - 1) / per_block;
    P.dual_blocks += D.blk_cnt;
    // chord steps of register-row inexact-Hessian classes in their own
    // kernel (fixed degrees: adaptive cells change class between steps)
    // (workgroup classes: one node per stand-in thread, so Q <= 256)
    D.chord = (D.prec & 2) && !P.adapt && D.count > 0 && !D.merged && (D.T == 0 || P.Q <= 256);
    if (D.chord) {
      // the chord kernel stages the modes of the cells it takes (its own and
      // those of classes merged into it), not the class's padded rows
      int modes = 0;
      for (int k = 0; k <= c; ++k)
        if (static_cast<int>((P.cls_map >> (4 * k)) & 15u) == c) modes = std::max(modes, P.cls_modes[k]);
      D.chord_kl = std::max(1, std::min(class_kl(P.M, P.kp, D.NP, D.T), modes));
      const int kl = D.chord_kl;
      auto lds_for = [&](int w) {
        return D.T > 0 ? chord_big_lds_bytes(P.M, D.T, P.Q, kl, w)
                       : chord_lds_bytes(P.M, D.NP, P.Q, kl, w);
      };
      D.chord_waves = 4;
      while (D.chord_waves > 1 && lds_for(D.chord_waves) > ctx->max_lds) D.chord_waves >>= 1;
      D.chord_lds = lds_for(D.chord_waves);
      if (D.chord_lds > ctx->max_lds) {
        D.chord = false;
      } else {
        D.cblk_off = P.dual_blocks;
        D.cblk_cnt = D.blk_cnt;
        P.dual_blocks += D.cblk_cnt;
      }
    }
  }
  P.dual_blocks = std::max(P.dual_blocks, 1);
  return IPM_OK;
}

DualParams dual_params(const Problem& P, int mode, int parity, const double* uhat, double* lam,
                       double* nodal, int cells, const int8_t* cellN, StepCtrl* ctrl,
                       unsigned long long* blk) {
  DualParams d{};
  d.blk_stats = blk;
  d.phi = P.d_phi;
  d.wphi = P.d_wphi;
  d.N = P.N;
  d.Q = P.Q;
  d.kp = P.kp;
  d.kl = P.kp;
  d.cells = cells;
  d.cellN = cellN;
  d.uhat = uhat;
  d.lam = lam;
  d.nodal = nodal;
  d.cp = P.cp;
  d.tau = P.tau;
  d.max_newton = P.max_newton;
  d.one_shot = mode == 0 ? P.one_shot : 0;
  d.mode = mode;
  d.dim = P.dim;
  d.ctrl = ctrl;
  d.parity = parity;
  // the other moments buffer holds the warm start the last update left
  if (mode == 0 && P.gwarm && uhat == P.d_u[parity]) {
    d.gwarm = P.d_u[parity ^ 1];
    d.s0 = P.d_s0;
  }
  return d;
}

// Newton kernel for size class c: over the class's lists of this step
// (list_mode) or over its cells in ascending order (setup, one-shot).  The
// ghosts' setup passes an explicit cell count with all N modes.
ipm_status launch_dual(ipm_ctx* ctx, const Problem& P, DualParams d, int c, bool list_mode,
                       int ghost_cells = -1) {
  const DualClass& D = P.cls[c];
  d.cls = c;
  d.bcache = D.bcache;
  d.kl = class_kl(P.M, P.kp, D.NP, D.T);
  int items;
  if (ghost_cells >= 0) {
    d.list_cap = 0;
    d.order = nullptr;
    d.cells = ghost_cells;
    items = ghost_cells;
  } else if (list_mode) {
    d.lists = D.d_lists + static_cast<size_t>(d.parity) * kSlots * D.cap;
    d.list_cap = D.cap;
    items = kSlots * D.cap;
    d.blk_stats = P.d_blk + kBlkStats * static_cast<size_t>(D.blk_off);
  } else {
    d.list_cap = 0;
    d.order = D.d_order;
    d.order_len = D.order_len;
    items = D.order_len;
    d.blk_stats = P.d_blk + kBlkStats * static_cast<size_t>(D.blk_off);
  }
  if (items == 0) return IPM_OK;
  // the inverse tiles belong to the problem's cells: the Dirichlet ghosts'
  // set-up runs the exact-Newton variant
  const int prec = ghost_cells >= 0 ? (D.prec & 1) : D.prec;
  if (prec & 2) P.set_hinv(d, D);
  bool pend = false;
  if (D.chord && ghost_cells < 0 && d.mode == 0) {
    // chord steps first (own block statistics), then the full kernel over
    // the cells they handed on
    DualParams dc = d;
    dc.kl = D.chord_kl;
    dc.blk_stats = P.d_blk + kBlkStats * static_cast<size_t>(D.cblk_off);
    dc.pend_list = D.d_pend;
    DualFn cf = D.T > 0 ? pick_big(P.M, D.T, 10) : pick_dual(P.M, D.NP, 10);
    if (!cf) return fail(ctx, IPM_E_ARG, "no chord kernel for this size");
    const int cpb = D.chord_waves * (D.T > 0 ? 1 : dual_cells_per_wave(P.M, D.NP));
    hipLaunchKernelGGL(cf, dim3((items + cpb - 1) / cpb), dim3(64 * D.chord_waves), D.chord_lds,
                       ctx->stream, dc);
    HIPCHK(ctx, hipGetLastError());
    d.pend = 1;
    d.pend_list = D.d_pend;
    d.reset_next = 0;
    pend = true;
  }
  if (D.T > 0) {
    DualFn fn = pick_big(P.M, D.T, prec);
    if (!fn) return fail(ctx, IPM_E_ARG, "no dual kernel for this size");
    hipLaunchKernelGGL(fn, dim3(pend ? kPendBlocks : items), dim3(256), D.lds, ctx->stream, d);
  } else {
    DualFn fn = pick_dual(P.M, D.NP, reg_variant(prec, 0, D.NP, P.Q));
    if (!fn) return fail(ctx, IPM_E_ARG, "no dual kernel for this size");
    const int per_block = D.waves * dual_cells_per_wave(P.M, D.NP);
    const int blocks = pend ? kPendBlocks : (items + per_block - 1) / per_block;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * D.waves), D.lds, ctx->stream, d);
  }
  HIPCHK(ctx, hipGetLastError());
  return IPM_OK;
}

// all Newton launches of one step or of the setup, class by class
ipm_status launch_dual_classes(ipm_ctx* ctx, const Problem& P, const DualParams& d, bool list_mode) {
  bool first = true;
  for (int c = 0; c < kCls; ++c) {
    if (P.cls[c].count == 0 || (list_mode && P.cls[c].merged)) continue;
    DualParams dc = d;
    dc.reset_next = first ? 1 : 0;
    first = false;
    ipm_status st = launch_dual(ctx, P, dc, c, list_mode);
    if (st != IPM_OK) return st;
  }
  return IPM_OK;
}

UpdateParams update_params(const Problem& P, int parity) {
  UpdateParams u{};
  u.wphi = P.d_wphi;
  u.N = P.N;
  u.Q = P.Q;
  u.kp = P.kp;
  u.cells = P.cells;
  u.nx = P.nx;
  u.ny = P.ny;
  u.dim = P.dim;
  u.cellN = P.d_cellN[parity];
  u.nodal = P.d_nodal;
  u.ghost = P.d_ghost;
  u.uold = P.d_u[parity];
  u.unew = P.d_u[parity ^ 1];
  u.gwarm = P.gwarm ? 1 : 0;
  u.stage_table = P.upd_stage ? 1 : 0;
  u.s0 = P.d_s0;
  u.res_part = P.d_res;
  for (int k = 0; k < 4; ++k) u.bc[k] = P.bc[k];
  u.flux = P.flux;
  u.gamma = P.cp.gamma;
  u.cfl = P.cfl;
  u.dx = P.dx;
  u.dy = P.dy;
  u.vol = P.vol;
  u.t_end = P.t_end;
  u.ctrl = P.d_ctrl;
  u.parity = parity;
  u.tau = P.tau;
  u.one_shot = P.one_shot;
  for (int c = 0; c < kCls; ++c) {
    const DualClass& D = P.cls[c];
    u.lists[c] = D.cap > 0 ? D.d_lists + static_cast<size_t>(parity ^ 1) * kSlots * D.cap : nullptr;
    u.list_cap[c] = D.cap;
  }
  u.adapt = P.adapt;
  u.p = P.p;
  u.deg_min = P.min_degree;
  u.deg_max = P.degree;
  u.delta_lo = P.delta_lo;
  u.delta_hi = P.delta_hi;
  u.cellN_next = P.adapt ? P.d_cellN[parity ^ 1] : nullptr;
  u.lam = P.d_lam;
  u.retard = P.d_retard;
  u.cls_map = P.cls_map;
  u.ctp = P.d_ctp;
  u.hinv_ok = P.adapt ? P.d_hinv_ok : nullptr;
  return u;
}

ipm_status enqueue_step(ipm_ctx* ctx, Problem& P) {
  const int parity = static_cast<int>(P.step_index & 1);
  DualParams d = dual_params(P, 0, parity, P.d_u[parity], P.d_lam, P.d_nodal, P.cells,
                             P.d_cellN[parity], P.d_ctrl, P.d_blk);
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
  if (ctx->timing) {
    while (ctx->ev.size() < ctx->ev_used + 4) {
      hipEvent_t e;
      HIPCHK(ctx, hipEventCreate(&e));
      ctx->ev.push_back(e);
    }
    e0 = ctx->ev[ctx->ev_used];
    e1 = ctx->ev[ctx->ev_used + 1];
    e2 = ctx->ev[ctx->ev_used + 2];
    e3 = ctx->ev[ctx->ev_used + 3];
    ctx->ev_used += 4;
    HIPCHK(ctx, hipEventRecord(e0, ctx->stream));
  }
  ipm_status st = launch_dual_classes(ctx, P, d, P.lists());
  if (st != IPM_OK) return st;
  if (ctx->timing) {
    HIPCHK(ctx, hipEventRecord(e1, ctx->stream));
    HIPCHK(ctx, hipEventRecord(e2, ctx->stream));
  }
  UpdateParams u = update_params(P, parity);
  UpdFn fn = pick_update(P.M, P.UG);
  hipLaunchKernelGGL(fn, dim3(P.upd_blocks), dim3(64 * P.upd_waves), P.upd_lds, ctx->stream, u);
  HIPCHK(ctx, hipGetLastError());
  if (ctx->timing) HIPCHK(ctx, hipEventRecord(e3, ctx->stream));
  if (P.steady_eps > 0.0) {
    hipLaunchKernelGGL(residual_kernel, dim3(1), dim3(256), 0, ctx->stream, P.d_ctrl, P.d_res,
                       P.upd_blocks, P.steady_eps, parity, P.d_blk, P.dual_blocks, 0, P.d_retard);
    HIPCHK(ctx, hipGetLastError());
  }
  ++P.step_index;
  return IPM_OK;
}

// residual of the last step and the Newton totals into the control block
ipm_status enqueue_close(ipm_ctx* ctx, Problem& P) {
  hipLaunchKernelGGL(residual_kernel, dim3(1), dim3(256), 0, ctx->stream, P.d_ctrl, P.d_res,
                     P.upd_blocks, P.steady_eps, static_cast<int>(P.step_index & 1), P.d_blk,
                     P.dual_blocks, 1, P.d_retard);
  HIPCHK(ctx, hipGetLastError());
  return IPM_OK;
}

// ---------------------------------------------------------------- batching

const void* pick_newton_batched(int M, int NP, int T, int prec = 0) {
  if (T > 0) {
    if (M == 1) return big_batched_pick<1>(T, prec);
    if (M == 4) return big_batched_pick<4>(T, prec);
    return nullptr;
  }
  if (M == 1) return dual_batched_pick<1>(NP, prec);
  if (M == 3) return dual_batched_pick<3>(NP, prec);
  if (M == 4) return dual_batched_pick<4>(NP, prec);
  return nullptr;
}

const void* pick_update_batched(int M, int G) {
  if (M == 1) return update_batched_pick<1>(G);
  if (M == 3) return update_batched_pick<3>(G);
  if (M == 4) return update_batched_pick<4>(G);
  return nullptr;
}

// Host part of a batch plan: the launch lists of both step parities for the
// problems `ids` (their next step and the one after) and the parameter and
// block-offset arrays the batched kernels read.
ipm_status plan_batch(ipm_ctx* ctx, const std::vector<int>& ids, BatchPlan& Bp,
                      std::vector<DualParams>& dps, std::vector<UpdateParams>& ups,
                      std::vector<int>& begins) {
  BatchPlan* B = &Bp;
  B->ids = ids;
  B->gen = ctx->gen;
  for (int id : ids) B->step0.push_back(get(ctx, id)->step_index);
  struct NEntry {
    DualParams d;
    int blocks;
    size_t lds;
  };
  struct UEntry {
    UpdateParams u;
    int blocks;
    size_t lds;
  };
  dps.clear();
  ups.clear();
  begins.clear();
  for (int ph = 0; ph < 2; ++ph) {
    std::map<std::string, std::vector<NEntry>> ng;
    std::map<std::string, std::pair<int, int>> nshape;  // key -> (threads, cells per block)
    std::map<std::string, std::array<int, 4>> nkind;    // key -> (M, lanes, workgroup, variant)
    std::map<std::string, const void*> nfn;
    std::map<std::string, std::vector<UEntry>> ug;
    std::map<std::string, const void*> ufn;
    std::map<std::string, int> uthreads;
    std::vector<BatchLaunch> resid;
    for (int id : ids) {
      Problem& P = *get(ctx, id);
      const int parity = static_cast<int>((P.step_index + ph) & 1);
      DualParams d = dual_params(P, 0, parity, P.d_u[parity], P.d_lam, P.d_nodal, P.cells,
                                 P.d_cellN[parity], P.d_ctrl, P.d_blk);
      bool first = true;
      for (int c = 0; c < kCls; ++c) {
        const DualClass& D = P.cls[c];
        if (D.count == 0 || (P.lists() && D.merged)) continue;
        DualParams dc = d;
        dc.cls = c;
        dc.bcache = D.bcache;
        dc.kl = class_kl(P.M, P.kp, D.NP, D.T);
        dc.reset_next = first ? 1 : 0;
        first = false;
        dc.blk_stats = P.d_blk + kBlkStats * static_cast<size_t>(D.blk_off);
        if (D.prec & 2) P.set_hinv(dc, D);
        int items;
        if (P.lists()) {
          dc.lists = D.d_lists + static_cast<size_t>(parity) * kSlots * D.cap;
          dc.list_cap = D.cap;
          items = kSlots * D.cap;
        } else {
          dc.list_cap = 0;
          dc.order = D.d_order;
          dc.order_len = D.order_len;
          items = D.order_len;
        }
        if (D.chord) {
          // stage 0: the chord kernel (own statistics); stage 1: the full
          // kernel over the cells it hands on
          DualParams dk = dc;
          dk.kl = D.chord_kl;
          dk.blk_stats = P.d_blk + kBlkStats * static_cast<size_t>(D.cblk_off);
          dk.pend_list = D.d_pend;
          const int cpb = D.chord_waves * (D.T > 0 ? 1 : dual_cells_per_wave(P.M, D.NP));
          const std::string ck = "0:" + std::to_string(P.M) + ":" + std::to_string(D.NP) + ":" +
                                 std::to_string(D.T) + ":" + std::to_string(64 * D.chord_waves);
          ng[ck].push_back({dk, (items + cpb - 1) / cpb, D.chord_lds});
          nshape[ck] = {64 * D.chord_waves, cpb};
          nkind[ck] = {P.M, D.NP, D.T > 0 ? 1 : 0, 10};
          nfn[ck] = pick_newton_batched(P.M, D.NP, D.T, 10);
          if (!nfn[ck]) return fail(ctx, IPM_E_ARG, "no batched chord kernel for this size");
          // pending mode: a fixed grid over the handed-on cells
          dc.pend = 1;
          dc.pend_list = D.d_pend;
          dc.reset_next = 0;
          dc.lists = nullptr;
          dc.list_cap = 0;
        }
        const int per_block = D.T > 0 ? 1 : D.waves * dual_cells_per_wave(P.M, D.NP);
        const int threads = D.T > 0 ? 256 : 64 * D.waves;
        const int kprec = reg_variant(D.prec, D.T, D.NP, P.Q);
        const std::string key = "1:" + std::to_string(P.M) + ":" + std::to_string(D.NP) + ":" +
                                std::to_string(D.T) + ":" + std::to_string(threads) + ":" +
                                std::to_string(kprec) + (dc.pend ? ":p" : "");
        ng[key].push_back({dc, dc.pend ? kPendBlocks : (items + per_block - 1) / per_block, D.lds});
        nshape[key] = {threads, per_block};
        nkind[key] = {P.M, D.NP, D.T > 0 ? 1 : 0, kprec};
        nfn[key] = pick_newton_batched(P.M, D.NP, D.T, kprec);
        if (!nfn[key]) return fail(ctx, IPM_E_ARG, "no batched dual kernel for this size");
      }
      const std::string ukey = std::to_string(P.M) + ":" + std::to_string(P.UG) + ":" +
                               std::to_string(P.upd_waves);
      ug[ukey].push_back({update_params(P, parity), P.upd_blocks, P.upd_lds});
      ufn[ukey] = pick_update_batched(P.M, P.UG);
      uthreads[ukey] = 64 * P.upd_waves;
      if (P.steady_eps > 0.0) {
        BatchLaunch L;
        L.kind = 2;
        L.pid = id;
        L.parity = parity;
        resid.push_back(L);
      }
    }
    for (auto& kv : ng) {  // keys "0:..." (chord stage) sort before "1:..."
      BatchLaunch L;
      L.kind = 0;
      L.stage = kv.first[0] == '0' ? 0 : 1;
      L.fn = nfn[kv.first];
      L.threads = nshape[kv.first].first;
      L.per_block = nshape[kv.first].second;
      L.M = nkind[kv.first][0];
      L.lanes = nkind[kv.first][1];
      L.workgroup = nkind[kv.first][2];
      L.variant = nkind[kv.first][3];
      L.lists = kv.second.front().d.list_cap > 0 || kv.second.front().d.lists != nullptr;
      L.pofs = dps.size();
      L.bofs = static_cast<int>(begins.size());
      L.n = static_cast<int>(kv.second.size());
      int acc = 0;
      for (const NEntry& e : kv.second) {
        dps.push_back(e.d);
        begins.push_back(acc);
        acc += e.blocks;
        L.lds = std::max(L.lds, e.lds);
      }
      begins.push_back(acc);
      L.blocks = acc;
      if (acc > 0) B->launches[ph].push_back(L);
    }
    for (auto& kv : ug) {
      BatchLaunch L;
      L.kind = 1;
      L.fn = ufn[kv.first];
      if (!L.fn) return fail(ctx, IPM_E_ARG, "no batched update kernel for this size");
      L.threads = uthreads[kv.first];
      L.pofs = ups.size();
      L.bofs = static_cast<int>(begins.size());
      L.n = static_cast<int>(kv.second.size());
      int acc = 0;
      for (const UEntry& e : kv.second) {
        ups.push_back(e.u);
        begins.push_back(acc);
        acc += e.blocks;
        L.lds = std::max(L.lds, e.lds);
      }
      begins.push_back(acc);
      L.blocks = acc;
      if (acc > 0) B->launches[ph].push_back(L);
    }
    for (const BatchLaunch& L : resid) B->launches[ph].push_back(L);
  }
  B->nd = dps.size();
  B->nu = ups.size();
  return IPM_OK;
}

// Build a batch plan in device buffers of its own: upload the parameter
// arrays and instantiate one graph per parity.
ipm_status add_graphs(ipm_ctx* ctx, BatchPlan& Bp);

// A batch plan: its launches and their parameter arrays on the device.  The
// graphs are added when the same plan is stepped a second time (add_graphs):
// a plan that changes every call (a serving loop admitting and finishing
// requests) runs launch by launch instead of paying two instantiations.
// prev (nullable): a retired plan of this context, idle on the device; its
// parameter arrays are taken over where they are large enough, so that a
// serving loop whose batch changes every round does not allocate and free
// (hipFree waits for the whole device) on every change.
ipm_status build_batch(ipm_ctx* ctx, const std::vector<int>& ids, std::unique_ptr<BatchPlan>& out,
                       BatchPlan* prev = nullptr) {
  auto B = std::make_unique<BatchPlan>();
  std::vector<DualParams> dps;
  std::vector<UpdateParams> ups;
  std::vector<int> begins;
  ipm_status pst = plan_batch(ctx, ids, *B, dps, ups, begins);
  if (pst != IPM_OK) return pst;
  if (prev && !prev->owned) prev = nullptr;
  auto take = [&](auto*& mine, auto*& theirs, size_t& cap, size_t theirs_cap, size_t need) {
    using T = std::remove_reference_t<decltype(*mine)>;
    need = std::max<size_t>(need, 1);
    if (prev && theirs && theirs_cap >= need) {
      mine = theirs;
      theirs = nullptr;
      cap = theirs_cap;
      return hipSuccess;
    }
    cap = need;
    return hipMalloc(reinterpret_cast<void**>(&mine), need * sizeof(T));
  };
  {
    size_t cap_b2 = 0;
    BatchPlan none;
    BatchPlan& pv = prev ? *prev : none;
    HIPCHK(ctx, take(B->d_dp, pv.d_dp, B->cap_dp, pv.cap_dp, dps.size()));
    HIPCHK(ctx, take(B->d_up, pv.d_up, B->cap_up, pv.cap_up, ups.size()));
    HIPCHK(ctx, take(B->d_begin, pv.d_begin, B->cap_begin, pv.cap_begin, begins.size()));
    HIPCHK(ctx, take(B->d_dev_begin, pv.d_dev_begin, cap_b2, pv.cap_begin, begins.size()));
    // both block-offset arrays hold cap_begin entries
    if (cap_b2 < B->cap_begin) B->cap_begin = cap_b2;
  }
  HIPCHK(ctx, hipMemcpyAsync(B->d_dp, dps.data(), dps.size() * sizeof(DualParams),
                             hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(B->d_up, ups.data(), ups.size() * sizeof(UpdateParams),
                             hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipMemcpyAsync(B->d_begin, begins.data(), begins.size() * sizeof(int),
                             hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  out = std::move(B);
  return IPM_OK;
}

ipm_status add_graphs(ipm_ctx* ctx, BatchPlan& Bp) {
  BatchPlan* B = &Bp;
  // one graph per parity: Newton launches in parallel, then the updates,
  // then the steady residuals
  for (int ph = 0; ph < 2; ++ph) {
    HIPCHK(ctx, hipGraphCreate(&B->graph[ph], 0));
    std::vector<hipGraphNode_t> newton, update, chords;
    for (const BatchLaunch& L : B->launches[ph]) {
      hipKernelNodeParams kp{};
      kp.gridDim = dim3(L.blocks);
      kp.blockDim = dim3(L.threads);
      kp.sharedMemBytes = static_cast<unsigned>(L.lds);
      kp.extra = nullptr;
      hipGraphNode_t node;
      if (L.kind == 0 || L.kind == 1) {
        const void* pp = L.kind == 0 ? static_cast<const void*>(B->d_dp + L.pofs)
                                     : static_cast<const void*>(B->d_up + L.pofs);
        const int* bg = (L.kind == 0 && L.lists) ? B->d_dev_begin + L.bofs : B->d_begin + L.bofs;
        int n = L.n;
        std::vector<hipGraphNode_t> deps;
        if (L.kind == 1) deps = newton;
        if (L.kind == 0 && L.stage == 1) deps = chords;
        if (L.kind == 0 && L.lists) {
          hipKernelNodeParams pk{};
          const DualParams* pdp = B->d_dp + L.pofs;
          int per_block = L.per_block;
          int* out = B->d_dev_begin + L.bofs;
          void* pargs[4] = {&pdp, &n, &per_block, &out};
          pk.func = reinterpret_cast<void*>(batch_prefix_kernel);
          pk.gridDim = dim3(1);
          pk.blockDim = dim3(64);
          pk.sharedMemBytes = 0;
          pk.kernelParams = pargs;
          pk.extra = nullptr;
          hipGraphNode_t pnode;
          HIPCHK(ctx, hipGraphAddKernelNode(&pnode, B->graph[ph], nullptr, 0, &pk));
          deps.push_back(pnode);
        }
        void* args[3] = {&pp, &bg, &n};
        kp.func = const_cast<void*>(L.fn);
        kp.kernelParams = args;
        HIPCHK(ctx, hipGraphAddKernelNode(&node, B->graph[ph], deps.data(), deps.size(), &kp));
        (L.kind == 0 ? newton : update).push_back(node);
        if (L.kind == 0 && L.stage == 0) chords.push_back(node);
      } else {
        const Problem& P = *get(ctx, L.pid);
        StepCtrl* C = P.d_ctrl;
        const double* rp = P.d_res;
        int nparts = P.upd_blocks;
        double eps = P.steady_eps;
        int par = L.parity;
        const unsigned long long* bs = P.d_blk;
        int nblk = P.dual_blocks, close = 0;
        Retard* R = P.d_retard;
        void* args[9] = {&C, &rp, &nparts, &eps, &par, &bs, &nblk, &close, &R};
        kp.func = reinterpret_cast<void*>(residual_kernel);
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(256);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        HIPCHK(ctx, hipGraphAddKernelNode(&node, B->graph[ph], update.data(), update.size(), &kp));
      }
    }
    HIPCHK(ctx, hipGraphInstantiate(&B->exec[ph], B->graph[ph], nullptr, nullptr, 0));
  }
  return IPM_OK;
}

bool batch_valid(const ipm_ctx* ctx, const BatchPlan* B, const std::vector<int>& ids) {
  if (!B || B->gen != ctx->gen || B->ids != ids) return false;
  for (size_t k = 0; k < ids.size(); ++k) {
    const Problem* P = ctx->problems[ids[k]].get();
    if (!P || P->step_index != B->step0[k] + B->steps_done) return false;
  }
  return true;
}

// One batched step of phase ph launch by launch on the context's stream;
// e (nullable): events around the Newton and the update phase.
ipm_status launch_batch_step(ipm_ctx* ctx, const BatchPlan& B, int ph, hipEvent_t* e) {
  if (e) HIPCHK(ctx, hipEventRecord(e[0], ctx->stream));
  int phase_kind = 0;
  for (const BatchLaunch& L : B.launches[ph]) {
    if (L.kind != 0 && phase_kind == 0) {
      if (e) {
        HIPCHK(ctx, hipEventRecord(e[1], ctx->stream));
        HIPCHK(ctx, hipEventRecord(e[2], ctx->stream));
      }
      phase_kind = 1;
    }
    if (L.kind == 0 || L.kind == 1) {
      const void* pp = L.kind == 0 ? static_cast<const void*>(B.d_dp + L.pofs)
                                   : static_cast<const void*>(B.d_up + L.pofs);
      const int* bg = (L.kind == 0 && L.lists) ? B.d_dev_begin + L.bofs : B.d_begin + L.bofs;
      int n = L.n;
      if (L.kind == 0 && L.lists) {
        hipLaunchKernelGGL(batch_prefix_kernel, dim3(1), dim3(64), 0, ctx->stream,
                           B.d_dp + L.pofs, n, L.per_block, B.d_dev_begin + L.bofs);
        HIPCHK(ctx, hipGetLastError());
      }
      void* args[3] = {&pp, &bg, &n};
      hipEvent_t* le = nullptr;
      if (e && L.kind == 0) {
        while (ctx->lev.size() < ctx->lev_used + 2) {
          hipEvent_t x;
          HIPCHK(ctx, hipEventCreate(&x));
          ctx->lev.push_back(x);
        }
        le = &ctx->lev[ctx->lev_used];
        ctx->lrec.push_back({L.M, L.lanes, L.workgroup, L.variant, L.threads, ctx->lev_used});
        ctx->lev_used += 2;
        HIPCHK(ctx, hipEventRecord(le[0], ctx->stream));
      }
      HIPCHK(ctx, hipLaunchKernel(L.fn, dim3(L.blocks), dim3(L.threads), args, L.lds, ctx->stream));
      if (le) HIPCHK(ctx, hipEventRecord(le[1], ctx->stream));
    } else {
      const Problem& P = *get(ctx, L.pid);
      hipLaunchKernelGGL(residual_kernel, dim3(1), dim3(256), 0, ctx->stream, P.d_ctrl, P.d_res,
                         P.upd_blocks, P.steady_eps, L.parity, P.d_blk, P.dual_blocks, 0,
                         P.d_retard);
      HIPCHK(ctx, hipGetLastError());
    }
  }
  if (e) HIPCHK(ctx, hipEventRecord(e[3], ctx->stream));
  return IPM_OK;
}

// `steps` batched steps: graph replays, or launch by launch with events
// around the Newton and update phases when kernel timing is on
ipm_status run_batch(ipm_ctx* ctx, BatchPlan& B, int steps) {
  for (int s = 0; s < steps; ++s) {
    const int ph = static_cast<int>(B.steps_done & 1);
    if (!ctx->timing && B.exec[ph]) {
      HIPCHK(ctx, hipGraphLaunch(B.exec[ph], ctx->stream));
    } else if (!ctx->timing) {
      ipm_status st = launch_batch_step(ctx, B, ph, nullptr);
      if (st != IPM_OK) return st;
    } else {
      while (ctx->ev.size() < ctx->ev_used + 4) {
        hipEvent_t e;
        HIPCHK(ctx, hipEventCreate(&e));
        ctx->ev.push_back(e);
      }
      hipEvent_t* e = &ctx->ev[ctx->ev_used];
      ctx->ev_used += 4;
      ipm_status st = launch_batch_step(ctx, B, ph, e);
      if (st != IPM_OK) return st;
    }
    ++B.steps_done;
    for (int id : B.ids) ++get(ctx, id)->step_index;
  }
  return IPM_OK;
}

ipm_status set_kernel_attributes(ipm_ctx* ctx) {
  static bool done = false;
  if (done) return IPM_OK;
  const int big = static_cast<int>(ctx->max_lds);
  // raise the dynamic LDS limit above the 64 KiB default (best effort)
  for (int M : {1, 3, 4})
    for (int NP : {8, 16, 32, 64})
      for (int prec : {0, 2, 4, 6, 10}) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(pick_dual(M, NP, prec)),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, big);
        (void)hipFuncSetAttribute(pick_newton_batched(M, NP, 0, prec),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, big);
      }
  for (int M : {1, 3, 4})
    for (int G : {16, 32, 64})
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(pick_update(M, G)),
                                hipFuncAttributeMaxDynamicSharedMemorySize, big);
  for (int M : {1, 4})
    for (int T : {1, 2, 4, 5, 6, 8, 9})
      for (int prec : {0, 1, 2, 3, 10}) {
        if ((prec & 1) && prec != 10 && T < 5) continue;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(pick_big(M, T, prec)),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, big);
        (void)hipFuncSetAttribute(pick_newton_batched(M, 16 * T, T, prec),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, big);
      }
  for (int M : {1, 3, 4}) {
    for (int NP : {8, 16, 32, 64})
      (void)hipFuncSetAttribute(pick_newton_batched(M, NP, 0),
                                hipFuncAttributeMaxDynamicSharedMemorySize, big);
    for (int G : {16, 32, 64})
      (void)hipFuncSetAttribute(pick_update_batched(M, G),
                                hipFuncAttributeMaxDynamicSharedMemorySize, big);
  }

  (void)hipGetLastError();  // the request is best effort; do not leave a sticky error
  done = true;
  return IPM_OK;
}

ipm_status validate(ipm_ctx* ctx, const ipm_problem* pb) {
  if (!pb) return fail(ctx, IPM_E_ARG, "problem is NULL");
  if (pb->equation < 0 || pb->equation > 2) return fail(ctx, IPM_E_ARG, "equation out of range");
  const int M = components(pb->equation);
  if (M == 1 && pb->entropy != IPM_ENT_QUADRATIC && pb->entropy != IPM_ENT_LOG_BARRIER)
    return fail(ctx, IPM_E_ARG, "Burgers needs the quadratic or the log-barrier entropy");
  if (M > 1 && pb->entropy != IPM_ENT_QUADRATIC && pb->entropy != IPM_ENT_EULER)
    return fail(ctx, IPM_E_ARG, "Euler needs the quadratic or the Euler entropy");
  if (pb->flux != IPM_FLUX_LF && pb->flux != IPM_FLUX_RUSANOV && pb->flux != IPM_FLUX_SG_ANALYTIC)
    return fail(ctx, IPM_E_ARG, "flux out of range");
  if (pb->flux == IPM_FLUX_SG_ANALYTIC) {
    if (pb->equation != IPM_BURGERS_1D || pb->entropy != IPM_ENT_QUADRATIC)
      return fail(ctx, IPM_E_ARG, "the analytic SG flux needs Burgers with the quadratic entropy");
    if (pb->bc[0] == IPM_BC_DIRICHLET || pb->bc[1] == IPM_BC_DIRICHLET || pb->adapt)
      return fail(ctx, IPM_E_ARG, "the analytic SG flux takes outflow or periodic boundaries and fixed degrees");
    if (pb->p >= 1 && pb->p <= 3 && pb->degree >= 0 && pb->degree <= 40 &&
        binom_basis(pb->p, pb->degree) > 16)
      return fail(ctx, IPM_E_ARG, "the analytic SG flux takes at most 16 basis functions");
  }
  if (pb->p < 1 || pb->p > 3) return fail(ctx, IPM_E_ARG, "p must be 1..3");
  if (pb->degree < 0 || pb->degree > 40) return fail(ctx, IPM_E_ARG, "degree must be 0..40");
  if (pb->quad_rule < IPM_QUAD_GAUSS_LEGENDRE || pb->quad_rule > IPM_QUAD_CC_SPARSE)
    return fail(ctx, IPM_E_ARG, "quad_rule out of range");
  if (pb->quad_rule != IPM_QUAD_CC_SPARSE && (pb->quad_per_dim < 1 || pb->quad_per_dim > 64))
    return fail(ctx, IPM_E_ARG, "quad_per_dim must be 1..64");
  if (pb->quad_rule == IPM_QUAD_CC_SPARSE && (pb->quad_per_dim < 0 || pb->quad_per_dim > 11))
    return fail(ctx, IPM_E_ARG, "the sparse-grid level must be 0..11");
  if (pb->precision < 0 || pb->precision > 2) return fail(ctx, IPM_E_ARG, "precision out of range");
  if (pb->precision == IPM_PREC_FP32)
    return fail(ctx, IPM_E_ARG,
                "IPM_PREC_FP32 is not provided: on this GPU FP32 vector arithmetic runs at the FP64 "
                "rate; use IPM_PREC_BF16 (split-BF16 MFMA Hessian)");
  if (!(pb->cfl > 0.0)) return fail(ctx, IPM_E_ARG, "cfl must be > 0");
  if (!(pb->tau > 0.0)) return fail(ctx, IPM_E_ARG, "tau must be > 0");
  if (pb->t_end < 0.0 || pb->steady_eps < 0.0)
    return fail(ctx, IPM_E_ARG, "t_end and steady_eps must be >= 0");
  if (pb->max_newton < 1) return fail(ctx, IPM_E_ARG, "max_newton must be >= 1");
  if (pb->nx < 1) return fail(ctx, IPM_E_ARG, "nx must be >= 1");
  if (pb->equation == IPM_EULER_2D && pb->ny < 1) return fail(ctx, IPM_E_ARG, "ny must be >= 1");
  if (!(pb->x1 > pb->x0)) return fail(ctx, IPM_E_ARG, "x1 must exceed x0");
  if (pb->equation == IPM_EULER_2D && !(pb->y1 > pb->y0))
    return fail(ctx, IPM_E_ARG, "y1 must exceed y0");
  if (M > 1 && !(pb->gamma > 1.0)) return fail(ctx, IPM_E_ARG, "gamma must be > 1");
  if (pb->entropy == IPM_ENT_LOG_BARRIER && !(pb->u_plus > pb->u_minus))
    return fail(ctx, IPM_E_ARG, "log-barrier needs u_minus < u_plus");
  const int sides = pb->equation == IPM_EULER_2D ? 4 : 2;
  for (int s = 0; s < sides; ++s)
    if (pb->bc[s] < 0 || pb->bc[s] > 2) return fail(ctx, IPM_E_ARG, "bc out of range");
  for (int s = 0; s < sides; s += 2)
    if ((pb->bc[s] == IPM_BC_PERIODIC) != (pb->bc[s + 1] == IPM_BC_PERIODIC))
      return fail(ctx, IPM_E_ARG, "periodic boundaries must be paired");
  bool any_dir = false;
  for (int s = 0; s < sides; ++s) any_dir |= pb->bc[s] == IPM_BC_DIRICHLET;
  if (any_dir && !pb->dirichlet) return fail(ctx, IPM_E_ARG, "Dirichlet sides need dirichlet states");
  if (!pb->ic_nodal && !pb->ic_moments) return fail(ctx, IPM_E_ARG, "need ic_nodal or ic_moments");
  if (pb->adapt) {
    if (pb->min_degree < 1 || pb->min_degree > pb->degree)
      return fail(ctx, IPM_E_ARG, "adaptivity needs 1 <= min_degree <= degree");
    if (!(pb->delta_lo <= pb->delta_hi))
      return fail(ctx, IPM_E_ARG, "adaptivity needs delta_lo <= delta_hi");
    if (pb->quad_rule != IPM_QUAD_GAUSS_LEGENDRE || pb->quad_per_dim < pb->degree + 1)
      return fail(ctx, IPM_E_ARG, "adaptivity needs the Gauss-Legendre rule with quad_per_dim >= degree + 1");
  }
  if (pb->hessian_reuse < 0 || pb->hessian_reuse > 2)
    return fail(ctx, IPM_E_ARG, "hessian_reuse must be 0, 1 or 2");
  if (!(pb->reuse_theta >= 0.0 && pb->reuse_theta < 1.0))
    return fail(ctx, IPM_E_ARG, "reuse_theta must be in [0, 1)");
  if (pb->n_retard != 0) {
    if (!pb->adapt || !(pb->steady_eps > 0.0))
      return fail(ctx, IPM_E_ARG, "refinement retardation needs adapt = 1 and steady_eps > 0");
    if (pb->n_retard < 0 || pb->n_retard > kMaxRetard || !pb->retard_degree || !pb->retard_eps)
      return fail(ctx, IPM_E_ARG, "refinement retardation needs 1..16 stages with degrees and tolerances");
    for (int k = 0; k < pb->n_retard; ++k) {
      const int dg = pb->retard_degree[k];
      if (dg < pb->min_degree || dg > pb->degree || (k > 0 && dg < pb->retard_degree[k - 1]))
        return fail(ctx, IPM_E_ARG, "retardation degrees must be non-decreasing in [min_degree, degree]");
    }
  }
  return IPM_OK;
}

}  // namespace

// The scalar fields at the head of a problem's control block (time, stop
// flags, status, step and Newton counters): what the host reads between
// steps, without the speed slots and list lengths behind them (96 KB).
constexpr size_t kCtrlHead = offsetof(StepCtrl, amax);

// The first fields of the control block alone (the serving loop's poll).
struct CtrlFlags {
  double t[2];
  int done[2];
  unsigned int status;
  unsigned int setup_status;
  unsigned long long steps;
};
static_assert(offsetof(CtrlFlags, done) == offsetof(StepCtrl, done) &&
                  offsetof(CtrlFlags, status) == offsetof(StepCtrl, status) &&
                  offsetof(CtrlFlags, steps) == offsetof(StepCtrl, steps),
              "CtrlFlags mirrors the head of StepCtrl");

// The serving loop's poll: the CtrlFlags heads of up to kPollBatch problems
// gathered into one contiguous device array (one 64-bit word per thread), so
// that a single device-to-host copy returns the flags of every active problem.
constexpr int kPollBatch = 64;
constexpr int kFlagWords = static_cast<int>(sizeof(CtrlFlags) / sizeof(unsigned long long));
static_assert(sizeof(CtrlFlags) % sizeof(unsigned long long) == 0, "CtrlFlags is whole words");
struct PollSources {
  const unsigned long long* src[kPollBatch];
};
__global__ __launch_bounds__(kPollBatch* kFlagWords) void poll_gather_kernel(PollSources ps, int n,
                                                                             unsigned long long* dst) {
  const int t = static_cast<int>(threadIdx.x);
  if (t < n * kFlagWords) dst[t] = ps.src[t / kFlagWords][t % kFlagWords];
}

// Device temporaries of one call: freed when the call returns, on every
// path, once the stream has drained.
struct TempBuffers {
  hipStream_t s;
  std::vector<void*> p;
  template <class T>
  hipError_t alloc(T** ptr, size_t bytes) {
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), bytes);
    if (e == hipSuccess) p.push_back(static_cast<void*>(*ptr));
    return e;
  }
  ~TempBuffers() {
    if (p.empty()) return;
    (void)hipStreamSynchronize(s);
    for (void* x : p) (void)hipFree(x);
  }
};

extern "C" {

const char* ipm_last_error(const ipm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int ipm_basis_size(int p, int degree) {
  if (p < 1 || degree < 0) return 0;
  return binom_basis(p, degree);
}

int ipm_quadrature_size(int rule, int p, int param) {
  if (p < 1 || p > 3 || rule < 0 || rule > 2) return 0;
  if (rule == IPM_QUAD_CC_SPARSE) {
    if (param < 0 || param > 11) return 0;
    std::vector<double> x, w;
    return cc_sparse_rule(p, param, x, w);
  }
  if (param < 1 || param > 64) return 0;
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= param;
  return Q;
}

ipm_status ipm_quadrature_rule(int rule, int p, int param, double* nodes, double* weights, int cap) {
  const int Q = ipm_quadrature_size(rule, p, param);
  if (Q == 0 || !nodes || !weights) return fail(nullptr, IPM_E_ARG, "ipm_quadrature_rule: bad arguments");
  if (Q > cap) return fail(nullptr, IPM_E_ARG, "ipm_quadrature_rule: capacity too small");
  std::vector<double> x, w;
  quadrature_rule(rule, p, param, x, w);
  std::memcpy(nodes, x.data(), sizeof(double) * Q * p);
  std::memcpy(weights, w.data(), sizeof(double) * Q);
  return IPM_OK;
}

ipm_status ipm_quadrature(int p, int quad_per_dim, double* nodes, double* weights, int cap) {
  if (p < 1 || p > 3 || quad_per_dim < 1 || quad_per_dim > 64 || !nodes || !weights)
    return fail(nullptr, IPM_E_ARG, "ipm_quadrature: bad arguments");
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= quad_per_dim;
  if (Q > cap) return fail(nullptr, IPM_E_ARG, "ipm_quadrature: capacity too small");
  std::vector<double> x, w;
  tensor_rule(p, quad_per_dim, x, w);
  std::memcpy(nodes, x.data(), sizeof(double) * Q * p);
  std::memcpy(weights, w.data(), sizeof(double) * Q);
  return IPM_OK;
}

// Host copy of the basis table Phi [Q][N] the library uploads (inspection).
ipm_status ipm_basis_table(int p, int degree, int quad_per_dim, double* Phi, int cap) {
  if (p < 1 || p > 3 || degree < 0 || quad_per_dim < 1 || quad_per_dim > 64 || !Phi)
    return fail(nullptr, IPM_E_ARG, "ipm_basis_table: bad arguments");
  std::vector<double> x, w;
  const int Q = tensor_rule(p, quad_per_dim, x, w);
  const int N = binom_basis(p, degree);
  if (static_cast<long long>(Q) * N > cap)
    return fail(nullptr, IPM_E_ARG, "ipm_basis_table: capacity too small");
  std::vector<double> t = basis_table(p, degree, Q, x);
  std::memcpy(Phi, t.data(), sizeof(double) * Q * N);
  return IPM_OK;
}

// stored inverses of the inexact-Hessian Newton: NP x NP doubles per cell
// (NP = 16T for the workgroup kernel; at least 16 for small cells, which
// may run on it), plus flags/slots
static size_t reuse_bytes(const ipm_problem* pb, int M, size_t cells) {
  // valid flags and slots; the chord kernels' warm-start <s_*> (Euler)
  size_t b = cells * (1 + sizeof(int)) + (pb->entropy == IPM_ENT_EULER ? cells * sizeof(double) : 0);
  if (pb->adapt) {  // one slot per cell of the largest class's size
    const int k = size_class(M * binom_basis(pb->p, pb->degree));
    const size_t np = k >= 4 ? 16 * class_tiles(k) : std::max(16, 8 << k);
    return b + cells * np * np * sizeof(float);
  }
  for (size_t c = 0; c < cells; ++c) {
    const int dg = pb->cell_degree ? pb->cell_degree[c] : pb->degree;
    const int n = M * binom_basis(pb->p, dg);
    const int k = size_class(n);
    const size_t np = k >= 4 ? 16 * class_tiles(k) : std::max(16, 8 << k);
    b += sizeof(float) * np * np;
  }
  return b;
}

size_t ipm_problem_footprint(const ipm_problem* pb) {
  if (!pb) return 0;
  const int M = components(pb->equation);
  const int N = binom_basis(pb->p, pb->degree);
  const int Q = std::max(1, ipm_quadrature_size(pb->quad_rule, pb->p, pb->quad_per_dim));
  const size_t cells = static_cast<size_t>(pb->nx) * (pb->equation == IPM_EULER_2D ? pb->ny : 1);
  const size_t n = static_cast<size_t>(M) * N;
  return sizeof(double) * (3 * cells * n + cells * Q * M + 2 * static_cast<size_t>(Q) * (N + 64) +
                           4 * static_cast<size_t>(Q) * M + cells / 8 + 64) +
         cells + 2 * (cells + static_cast<size_t>(kCls) * kSlots * 16) * sizeof(int) + cells * sizeof(int) +
         sizeof(StepCtrl) +
         (pb->adapt ? cells + static_cast<size_t>(pb->degree) * 2 * (cells + kSlots * 16) * sizeof(int)
                    : 0) +
         (pb->hessian_reuse ? reuse_bytes(pb, M, cells) : 0);
}

ipm_status ipm_create(const ipm_config* cfg, ipm_ctx** out) {
  if (!cfg || !out) return fail(nullptr, IPM_E_ARG, "ipm_create: NULL argument");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(nullptr, IPM_E_DEVICE, "ipm_create: no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev) return fail(nullptr, IPM_E_ARG, "ipm_create: bad device");
  auto ctx = std::make_unique<ipm_ctx>();
  ctx->device = cfg->device;
  ctx->budget = cfg->hbm_budget_bytes;
  ctx->max_problems = cfg->max_problems > 0 ? cfg->max_problems : 1024;
  e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return fail(nullptr, IPM_E_DEVICE, hipGetErrorString(e));
  ctx->stream = static_cast<hipStream_t>(cfg->hip_stream);  // NULL: the null stream
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, cfg->device) ==
          hipSuccess &&
      lds > 0)
    ctx->max_lds = static_cast<size_t>(lds);
  (void)hipGetLastError();
  if (set_kernel_attributes(ctx.get()) != IPM_OK) return fail(nullptr, IPM_E_DEVICE, ctx->err);
  {
    // the static scratch's address on this device (current), once per device
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot& slot = g_scratch[cfg->device];
    if (!slot.ptr) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(nullptr, IPM_E_DEVICE,
                    std::string("ipm_create: static scratch address: ") + hipGetErrorString(e));
      slot.ptr = static_cast<unsigned char*>(ptr);
    }
    ctx->scratch = slot.ptr;
  }
  *out = ctx.release();
  return IPM_OK;
}

ipm_status ipm_destroy(ipm_ctx* ctx) {
  if (!ctx) return IPM_E_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->batch.reset();
  ctx->static_plan.reset();
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot& slot = g_scratch[ctx->device];
    if (slot.owner == ctx) slot.owner = nullptr;
  }
  for (auto& p : ctx->problems) free_problem(p.get());
  for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->lev) (void)hipEventDestroy(e);
  if (ctx->d_poll) (void)hipFree(ctx->d_poll);
  if (ctx->h_poll) (void)hipHostFree(ctx->h_poll);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return IPM_OK;
}

ipm_status ipm_set_problem(ipm_ctx* ctx, const ipm_problem* pb, int* problem_id) {
  if (!ctx || !problem_id) return fail(ctx, IPM_E_ARG, "NULL argument");
  ipm_status st = validate(ctx, pb);
  if (st != IPM_OK) return st;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  auto up = std::make_unique<Problem>();
  Problem& P = *up;
  P.eq = pb->equation;
  P.M = components(pb->equation);
  P.dim = pb->equation == IPM_EULER_2D ? 2 : 1;
  P.p = pb->p;
  P.degree = pb->degree;
  P.N = binom_basis(pb->p, pb->degree);
  std::vector<double> nodes, w;
  P.Q = quadrature_rule(pb->quad_rule, pb->p, pb->quad_per_dim, nodes, w);
  P.nx = pb->nx;
  P.ny = P.dim == 2 ? pb->ny : 1;
  P.cells = P.nx * P.ny;
  P.flux = pb->flux;
  P.max_newton = pb->max_newton;
  P.one_shot = pb->one_shot ? 1 : 0;
  P.precision = pb->precision;
  for (int k = 0; k < 4; ++k) P.bc[k] = (P.dim == 1 && k >= 2) ? IPM_BC_OUTFLOW : pb->bc[k];
  P.cfl = pb->cfl;
  P.t_end = pb->t_end;
  P.tau = pb->tau;
  P.steady_eps = pb->steady_eps;
  P.dx = (pb->x1 - pb->x0) / pb->nx;
  P.dy = P.dim == 2 ? (pb->y1 - pb->y0) / pb->ny : 1.0;
  P.vol = P.dim == 2 ? P.dx * P.dy : P.dx;
  P.cp.entropy = pb->entropy;
  P.cp.gamma = pb->gamma;
  P.cp.r1mg = 1.0 / (1.0 - pb->gamma);
  P.cp.g75 = pb->gamma == 1.4 ? 1 : 0;
  P.cp.um = pb->u_minus;
  P.cp.up = pb->u_plus;
  P.cp.log_range = pb->entropy == IPM_ENT_LOG_BARRIER ? std::log(pb->u_plus - pb->u_minus) : 0.0;
  P.adapt = pb->adapt ? 1 : 0;
  P.hessian_reuse = pb->hessian_reuse;
  P.reuse_theta = pb->reuse_theta > 0.0 ? pb->reuse_theta : 0.5;
  P.min_degree = pb->min_degree;
  P.delta_lo = pb->delta_lo;
  P.delta_hi = pb->delta_hi;
  std::vector<int8_t> cellN;
  int counts[kCls] = {};
  std::vector<int> cell_cls;
  const int lo_deg = P.adapt ? P.min_degree : 0;
  if (pb->cell_degree || P.adapt) {
    cellN.resize(P.cells);
    cell_cls.resize(P.cells);
    for (int c = 0; c < P.cells; ++c) {
      const int dg = pb->cell_degree ? pb->cell_degree[c] : pb->degree;
      if (dg < lo_deg || dg > pb->degree) return fail(ctx, IPM_E_ARG, "cell_degree out of range");
      cellN[c] = static_cast<int8_t>(binom_basis(pb->p, dg));
      cell_cls[c] = size_class(cellN[c] * P.M);
      ++counts[cell_cls[c]];
      P.cls_modes[cell_cls[c]] = std::max(P.cls_modes[cell_cls[c]], static_cast<int>(cellN[c]));
    }
    P.uneven = true;
  } else {
    counts[size_class(P.M * P.N)] = P.cells;
    P.cls_modes[size_class(P.M * P.N)] = P.N;
  }
  int plan_counts[kCls];
  for (int c = 0; c < kCls; ++c) plan_counts[c] = counts[c];
  if (P.adapt)  // every level may hold every cell
    for (int dg = P.min_degree; dg <= P.degree; ++dg)
      plan_counts[size_class(binom_basis(pb->p, dg) * P.M)] = P.cells;
  st = plan(ctx, P, plan_counts);
  if (st != IPM_OK) return st;
  for (int c = 0; c < kCls; ++c) P.cls[c].order_len = counts[c];
  {
    // unknowns per launching class (cells of a merged class run in the
    // larger class's launch): the range over its cells, or over every level
    // for adaptive problems
    auto note = [&](int c, int n) {
      int t = static_cast<int>((P.cls_map >> (4 * c)) & 15u);
      DualClass& D = P.cls[t];
      D.n_min = D.n_min == 0 ? n : std::min(D.n_min, n);
      D.n_max = std::max(D.n_max, n);
    };
    if (P.adapt) {
      for (int dg = P.min_degree; dg <= P.degree; ++dg) {
        const int n = binom_basis(pb->p, dg) * P.M;
        note(size_class(n), n);
      }
    } else if (!cellN.empty()) {
      for (int c = 0; c < P.cells; ++c) note(cell_cls[c], cellN[c] * P.M);
    } else {
      note(size_class(P.M * P.N), P.M * P.N);
    }
  }

  const size_t fp = ipm_problem_footprint(pb);
  if (ctx->budget && ctx->used + fp > ctx->budget)
    return fail(ctx, IPM_E_NOMEM, "problem does not fit the HBM budget");
  int slot = -1;
  for (size_t k = 0; k < ctx->problems.size(); ++k)
    if (!ctx->problems[k]) {
      slot = static_cast<int>(k);
      break;
    }
  if (slot < 0) {
    if (static_cast<int>(ctx->problems.size()) >= ctx->max_problems)
      return fail(ctx, IPM_E_BUSY, "no free problem slot");
    ctx->problems.emplace_back();
    slot = static_cast<int>(ctx->problems.size()) - 1;
  }

  // tables: Phi and w*Phi, zero padded to kp columns
  const std::vector<double> phi = basis_table(pb->p, pb->degree, P.Q, nodes);
  std::vector<double> phip(static_cast<size_t>(P.Q) * P.kp, 0.0), wphip(phip.size(), 0.0);
  for (int q = 0; q < P.Q; ++q)
    for (int i = 0; i < P.N; ++i) {
      phip[static_cast<size_t>(q) * P.kp + i] = phi[static_cast<size_t>(q) * P.N + i];
      wphip[static_cast<size_t>(q) * P.kp + i] = w[q] * phi[static_cast<size_t>(q) * P.N + i];
    }
  const size_t cn = static_cast<size_t>(P.cells) * P.M * P.N;
  const size_t nod = static_cast<size_t>(P.cells) * P.Q * P.M;
  auto alloc = [&](void** ptr, size_t bytes) -> hipError_t {
    P.bytes += bytes;
    return hipMalloc(ptr, std::max<size_t>(bytes, 8));
  };
  auto cleanup = [&](ipm_status s) {
    free_problem(&P);
    return s;
  };
#define ALLOC(ptr, bytes)                                                        \
  do {                                                                           \
    if (alloc(reinterpret_cast<void**>(&(ptr)), (bytes)) != hipSuccess)          \
      return cleanup(fail(ctx, IPM_E_NOMEM, "device allocation failed"));        \
  } while (0)
  ALLOC(P.d_phi, phip.size() * sizeof(double));
  ALLOC(P.d_wphi, wphip.size() * sizeof(double));
  ALLOC(P.d_u[0], cn * sizeof(double));
  ALLOC(P.d_u[1], cn * sizeof(double));
  ALLOC(P.d_lam, cn * sizeof(double));
  ALLOC(P.d_nodal, nod * sizeof(double));
  ALLOC(P.d_ghost, 4 * static_cast<size_t>(P.Q) * P.M * sizeof(double));
  ALLOC(P.d_res, static_cast<size_t>(P.upd_blocks) * sizeof(double));
  ALLOC(P.d_blk, static_cast<size_t>(P.dual_blocks) * kBlkStats * sizeof(unsigned long long));
  for (DualClass& D : P.cls) {
    if (D.cap > 0) ALLOC(D.d_lists, 2 * static_cast<size_t>(kSlots) * D.cap * sizeof(int));
    if (D.chord) ALLOC(D.d_pend, static_cast<size_t>(D.count) * sizeof(int));
    if (P.uneven && D.order_len > 0) ALLOC(D.d_order, static_cast<size_t>(D.order_len) * sizeof(int));
  }
  ALLOC(P.d_ctrl, sizeof(StepCtrl));
  P.gwarm = false;
  if (P.cp.entropy == kEntEuler && !P.adapt)
    for (const DualClass& D : P.cls) P.gwarm = P.gwarm || D.chord;
  if (P.gwarm) ALLOC(P.d_s0, static_cast<size_t>(P.cells) * sizeof(double));
  if (pb->n_retard > 0) ALLOC(P.d_retard, sizeof(Retard));
  if (P.flux == IPM_FLUX_SG_ANALYTIC)
    ALLOC(P.d_ctp, static_cast<size_t>(P.N) * P.N * P.N * sizeof(double));
  if (P.hessian_reuse && P.adapt) {
    // one slot per cell, sized for the largest inexact-Hessian class
    int npmax = 0;
    for (DualClass& D : P.cls)
      if (D.configured && (D.prec & 2)) npmax = std::max(npmax, D.NP);
    if (npmax > 0) {
      P.hinv_all_stride = static_cast<long long>(npmax) * npmax;
      ALLOC(P.d_hinv_all, static_cast<size_t>(P.cells) * P.hinv_all_stride * sizeof(float));
      ALLOC(P.d_hinv_ok, static_cast<size_t>(P.cells));
    }
  } else if (P.hessian_reuse) {
    // NP x NP doubles for the cells of each inexact-Hessian class only
    bool any = false;
    for (DualClass& D : P.cls)
      if (D.configured && (D.prec & 2) && D.order_len > 0) {
        ALLOC(D.d_hinv, static_cast<size_t>(D.order_len) * D.NP * D.NP * sizeof(float));
        any = true;
      }
    if (any) {
      ALLOC(P.d_hinv_ok, static_cast<size_t>(P.cells));
      if (P.uneven) ALLOC(P.d_hinv_slot, static_cast<size_t>(P.cells) * sizeof(int));
    }
  }
  if (P.uneven) ALLOC(P.d_cellN[0], static_cast<size_t>(P.cells));
  if (P.adapt) ALLOC(P.d_cellN[1], static_cast<size_t>(P.cells));
  else P.d_cellN[1] = P.d_cellN[0];
#undef ALLOC
  hipStream_t s = ctx->stream;
#define CHK(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return cleanup(fail(ctx, IPM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  CHK(hipMemcpyAsync(P.d_phi, phip.data(), phip.size() * sizeof(double), hipMemcpyHostToDevice, s));
  CHK(hipMemcpyAsync(P.d_wphi, wphip.data(), wphip.size() * sizeof(double), hipMemcpyHostToDevice, s));
  std::vector<std::vector<int>> orders(kCls);
  if (P.uneven) {
    CHK(hipMemcpyAsync(P.d_cellN[0], cellN.data(), cellN.size(), hipMemcpyHostToDevice, s));
    if (P.adapt)
      CHK(hipMemcpyAsync(P.d_cellN[1], cellN.data(), cellN.size(), hipMemcpyHostToDevice, s));
    for (int c = 0; c < P.cells; ++c) orders[cell_cls[c]].push_back(c);
    for (int k = 0; k < kCls; ++k)
      if (P.cls[k].d_order)
        CHK(hipMemcpyAsync(P.cls[k].d_order, orders[k].data(), orders[k].size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
  }
  CHK(hipMemsetAsync(P.d_ctrl, 0, sizeof(StepCtrl), s));
  // modes above a cell's fixed level stay zero in both moment buffers (the
  // update writes only the cell's own modes; set-up fills buffer 0)
  CHK(hipMemsetAsync(P.d_u[1], 0, cn * sizeof(double), s));
  if (P.d_hinv_ok) CHK(hipMemsetAsync(P.d_hinv_ok, 0, static_cast<size_t>(P.cells), s));
  std::vector<int> hslot;
  if (P.d_hinv_slot) {  // a cell's slot: its position in its class's cell order
    hslot.assign(P.cells, 0);
    std::vector<int> seen(kCls, 0);
    for (int c = 0; c < P.cells; ++c) hslot[c] = seen[cell_cls[c]]++;
    CHK(hipMemcpyAsync(P.d_hinv_slot, hslot.data(), hslot.size() * sizeof(int),
                       hipMemcpyHostToDevice, s));
  }
  std::vector<double> ctp;
  if (P.d_ctp) {
    // App. A: C_i = <phi phi^T phi_i>; the integrands have degree <= 3M, so a
    // tensor Gauss-Legendre rule of 3M/2 + 1 points per dimension is exact
    std::vector<double> cn, cw;
    const int cq = tensor_rule(pb->p, (3 * pb->degree) / 2 + 1, cn, cw);
    const std::vector<double> cphi = basis_table(pb->p, pb->degree, cq, cn);
    const int N = P.N;
    ctp.assign(static_cast<size_t>(N) * N * N, 0.0);
    for (int q = 0; q < cq; ++q)
      for (int i = 0; i < N; ++i) {
        const double wi = cw[q] * cphi[static_cast<size_t>(q) * N + i];
        for (int a = 0; a < N; ++a) {
          const double wia = wi * cphi[static_cast<size_t>(q) * N + a];
          for (int b = 0; b < N; ++b)
            ctp[(static_cast<size_t>(i) * N + a) * N + b] += wia * cphi[static_cast<size_t>(q) * N + b];
        }
      }
    CHK(hipMemcpyAsync(P.d_ctp, ctp.data(), ctp.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  Retard hr{};
  if (P.d_retard) {
    hr.n = pb->n_retard;
    for (int k = 0; k < hr.n; ++k) {
      hr.deg[k] = pb->retard_degree[k];
      hr.eps[k] = pb->retard_eps[k];
    }
    CHK(hipMemcpyAsync(P.d_retard, &hr, sizeof(Retard), hipMemcpyHostToDevice, s));
  }
  // one-shot over work lists (adaptive): the first step's lists hold every
  // cell, by its initial size class, spread over the slots
  std::vector<std::vector<int>> first_lists(kCls);
  std::vector<unsigned> first_len(static_cast<size_t>(kCls) * kSlots, 0u);
  if (P.one_shot && P.lists()) {
    for (int c = 0; c < P.cells; ++c) {
      const int k = static_cast<int>((P.cls_map >> (4 * cell_cls[c])) & 15u);
      const DualClass& D = P.cls[k];
      std::vector<int>& L = first_lists[k];
      if (L.empty()) L.assign(static_cast<size_t>(kSlots) * D.cap, -1);
      const int slot = (c / std::max(1, (P.cells + kSlots - 1) / kSlots)) % kSlots;
      unsigned& len = first_len[static_cast<size_t>(k) * kSlots + slot];
      if (static_cast<int>(len) >= D.cap) return cleanup(fail(ctx, IPM_E_ARG, "work list overflow"));
      L[static_cast<size_t>(slot) * D.cap + len++] = c;
    }
    for (int k = 0; k < kCls; ++k)
      if (!first_lists[k].empty())
        CHK(hipMemcpyAsync(P.cls[k].d_lists, first_lists[k].data(),
                           first_lists[k].size() * sizeof(int), hipMemcpyHostToDevice, s));
    std::vector<unsigned> lens(sizeof(StepCtrl::list_len) / sizeof(unsigned), 0u);
    for (int k = 0; k < kCls; ++k)
      for (int sl = 0; sl < kSlots; ++sl)
        lens[list_len_index(0, k, sl)] = first_len[static_cast<size_t>(k) * kSlots + sl];
    CHK(hipMemcpyAsync(&P.d_ctrl->list_len[0], lens.data(), lens.size() * sizeof(unsigned),
                       hipMemcpyHostToDevice, s));
  }
  CHK(hipMemsetAsync(P.d_blk, 0, static_cast<size_t>(P.dual_blocks) * kBlkStats * sizeof(unsigned long long), s));
  CHK(hipMemsetAsync(P.d_res, 0, static_cast<size_t>(P.upd_blocks) * sizeof(double), s));
  CHK(hipMemsetAsync(P.d_ghost, 0, 4 * static_cast<size_t>(P.Q) * P.M * sizeof(double), s));
  CHK(hipMemsetAsync(P.d_nodal, 0, nod * sizeof(double), s));

  // staging of the host inputs (freed on every return, after the stream
  // has drained)
  TempBuffers staging{s, {}};
  double* d_in = nullptr;
  double* d_dual = nullptr;
  const size_t in_len = pb->ic_nodal ? nod : cn;
  CHK(staging.alloc(&d_in, in_len * sizeof(double)));
  CHK(hipMemcpyAsync(d_in, pb->ic_nodal ? pb->ic_nodal : pb->ic_moments, in_len * sizeof(double),
                     hipMemcpyHostToDevice, s));
  if (pb->ic_dual) {
    CHK(staging.alloc(&d_dual, cn * sizeof(double)));
    CHK(hipMemcpyAsync(d_dual, pb->ic_dual, cn * sizeof(double), hipMemcpyHostToDevice, s));
  }
  SetupParams sp{};
  sp.wphi = P.d_wphi;
  sp.N = P.N;
  sp.Q = P.Q;
  sp.kp = P.kp;
  sp.cells = P.cells;
  sp.cellN = P.d_cellN[0];
  sp.ic_nodal = pb->ic_nodal ? d_in : nullptr;
  sp.ic_moments = pb->ic_nodal ? nullptr : d_in;
  sp.ic_dual = d_dual;
  sp.uhat = P.d_u[0];
  sp.lam = P.d_lam;
  sp.cp = P.cp;
  sp.status = &P.d_ctrl->setup_status;
  {
    const size_t total = cn;
    const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
    if (blocks) hipLaunchKernelGGL(pick_setup(P.M), dim3(blocks), dim3(256), 0, s, sp);
    CHK(hipGetLastError());
  }
  // converge the initial dual (setup mode of the dual kernel)
  {
    DualParams d = dual_params(P, 1, 0, P.d_u[0], P.d_lam, P.d_nodal, P.cells, P.d_cellN[0], P.d_ctrl,
                               P.d_blk);
    st = launch_dual_classes(ctx, P, d, false);
    if (st != IPM_OK) return cleanup(st);
  }
  // Dirichlet ghosts: fixed moments, converged dual, their nodal ansatz and speeds
  int dsides[4], nd = 0;
  for (int k = 0; k < 4; ++k)
    if (P.bc[k] == IPM_BC_DIRICHLET) dsides[nd++] = k;
  double gax = 0.0, gay = 0.0;
  if (nd > 0) {
    const size_t gq = static_cast<size_t>(P.Q) * P.M;
    std::vector<double> gin(nd * gq);
    for (int k = 0; k < nd; ++k)
      std::memcpy(&gin[k * gq], pb->dirichlet + dsides[k] * gq, gq * sizeof(double));
    TempBuffers gtemps{s, {}};  // the ghosts' temporaries, freed on every return
    double *d_gin = nullptr, *d_gu = nullptr, *d_gl = nullptr, *d_gn = nullptr;
    StepCtrl* d_gc = nullptr;
    unsigned long long* d_gb = nullptr;
    CHK(gtemps.alloc(&d_gb, 64 * sizeof(unsigned long long)));
    CHK(hipMemsetAsync(d_gb, 0, 64 * sizeof(unsigned long long), s));
    CHK(gtemps.alloc(&d_gin, gin.size() * sizeof(double)));
    CHK(gtemps.alloc(&d_gu, nd * static_cast<size_t>(P.M) * P.N * sizeof(double)));
    CHK(gtemps.alloc(&d_gl, nd * static_cast<size_t>(P.M) * P.N * sizeof(double)));
    CHK(gtemps.alloc(&d_gn, gin.size() * sizeof(double)));
    CHK(gtemps.alloc(&d_gc, sizeof(StepCtrl)));
    CHK(hipMemsetAsync(d_gc, 0, sizeof(StepCtrl), s));
    CHK(hipMemcpyAsync(d_gin, gin.data(), gin.size() * sizeof(double), hipMemcpyHostToDevice, s));
    SetupParams gp = sp;
    gp.cells = nd;
    gp.cellN = nullptr;
    gp.ic_nodal = d_gin;
    gp.ic_moments = nullptr;
    gp.ic_dual = nullptr;
    gp.uhat = d_gu;
    gp.lam = d_gl;
    gp.status = &d_gc->setup_status;
    hipLaunchKernelGGL(pick_setup(P.M), dim3(1), dim3(256), 0, s, gp);
    CHK(hipGetLastError());
    DualParams d1 = dual_params(P, 1, 0, d_gu, d_gl, d_gn, nd, nullptr, d_gc, d_gb);
    st = launch_dual(ctx, P, d1, P.full_cls, false, nd);
    if (st != IPM_OK) return cleanup(st);
    for (int k = 0; k < nd; ++k)
      CHK(hipMemcpyAsync(P.d_ghost + dsides[k] * gq, d_gn + k * gq, gq * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
    StepCtrl gc;
    CHK(hipMemcpyAsync(&gc, d_gc, sizeof(StepCtrl), hipMemcpyDeviceToHost, s));
    CHK(hipStreamSynchronize(s));
    if (gc.setup_status || gc.status)
      return cleanup(fail(ctx, IPM_E_REALIZABILITY, "Dirichlet ghost state has no admissible dual"));
    for (int k = 0; k < kSlots; ++k) {
      gax = std::max(gax, __builtin_bit_cast(double, gc.amax[0][0][k * kSlotStride]));
      gay = std::max(gay, __builtin_bit_cast(double, gc.amax[0][1][k * kSlotStride]));
    }
  }
  StepCtrl hc;
  CHK(hipMemcpyAsync(&hc, P.d_ctrl, sizeof(StepCtrl), hipMemcpyDeviceToHost, s));
  CHK(hipStreamSynchronize(s));
  if (hc.setup_status) {
    std::string why = (hc.setup_status & kStRealizability) ? "initial state outside the entropy's domain"
                      : (hc.setup_status & kStNewton)      ? "initial dual did not converge"
                                                           : "initial dual solve failed";
    return cleanup(fail(ctx, hc.setup_status & kStRealizability ? IPM_E_REALIZABILITY : IPM_E_NEWTON,
                        why + " (status " + std::to_string(hc.setup_status) + ")"));
  }
  // keep the speed slots of the converged initial state (the first step of
  // the classical mode starts there); one-shot recomputes every cell's ansatz
  if (P.one_shot) CHK(hipMemsetAsync(&P.d_ctrl->amax[0][0][0], 0, sizeof(P.d_ctrl->amax[0]), s));
  const double gam[2] = {gax, gay};
  CHK(hipMemcpyAsync(&P.d_ctrl->ghost_amax[0], gam, sizeof(gam), hipMemcpyHostToDevice, s));
  CHK(hipStreamSynchronize(s));
#undef CHK
  P.charged = std::max(fp, P.bytes);
  // the estimate admitted the problem; the allocation it made is what counts
  if (ctx->budget && ctx->used + P.charged > ctx->budget)
    return cleanup(fail(ctx, IPM_E_NOMEM, "problem does not fit the HBM budget (allocated " +
                                              std::to_string(P.bytes) + " bytes)"));
  ctx->used += P.charged;
  ++ctx->gen;
  ctx->problems[slot] = std::move(up);
  *problem_id = slot;
  return IPM_OK;
}

ipm_status ipm_step(ipm_ctx* ctx, int n_ids, const int* ids, int max_steps, ipm_step_info* info) {
  if (!ctx) return IPM_E_ARG;
  if (n_ids < 0 || (n_ids > 0 && !ids) || max_steps < 0)
    return fail(ctx, IPM_E_ARG, "ipm_step: bad arguments");
  for (int k = 0; k < n_ids; ++k)
    if (!get(ctx, ids[k])) return fail(ctx, IPM_E_STATE, "ipm_step: unknown problem id");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  // one problem whose cells span several Newton kernel shapes also steps
  // through a graph, so that those launches overlap instead of queueing
  bool graph_one = false;
  if (n_ids == 1 && max_steps > 0) {
    int shapes = 0;
    for (const DualClass& D : get(ctx, ids[0])->cls) shapes += (D.count > 0 && !D.merged) ? 1 : 0;
    graph_one = shapes >= 2;
  }
  if ((n_ids >= 2 || graph_one) && max_steps > 0) {
    // several problems: batched launches per kernel shape, replayed as graphs
    std::vector<int> v(ids, ids + n_ids);
    for (size_t a = 0; a < v.size(); ++a)
      for (size_t b = a + 1; b < v.size(); ++b)
        if (v[a] == v[b]) return fail(ctx, IPM_E_ARG, "ipm_step: repeated problem id");
    if (!batch_valid(ctx, ctx->batch.get(), v)) {
      // the old plan's graphs may still be queued: drain before freeing
      if (ctx->batch) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      std::unique_ptr<BatchPlan> retired = std::move(ctx->batch);
      ipm_status st = build_batch(ctx, v, ctx->batch, retired.get());
      if (st != IPM_OK) return st;
    } else if (!ctx->batch->exec[0]) {
      ipm_status st = add_graphs(ctx, *ctx->batch);  // the plan is stepped again: replay it
      if (st != IPM_OK) return st;
    }
    ipm_status st = run_batch(ctx, *ctx->batch, max_steps);
    if (st != IPM_OK) return st;
  } else {
    for (int s = 0; s < max_steps; ++s)
      for (int k = 0; k < n_ids; ++k) {
        ipm_status st = enqueue_step(ctx, *get(ctx, ids[k]));
        if (st != IPM_OK) return st;
      }
  }
  if (max_steps > 0)
    for (int k = 0; k < n_ids; ++k) {
      ipm_status st = enqueue_close(ctx, *get(ctx, ids[k]));
      if (st != IPM_OK) return st;
    }
  if (info)
    for (int k = 0; k < n_ids; ++k) {
      ipm_status st = ipm_query(ctx, ids[k], &info[k]);
      if (st != IPM_OK) return st;
    }
  return IPM_OK;
}

ipm_status ipm_step_static(ipm_ctx* ctx, int n_ids, const int* ids, int max_steps,
                           ipm_step_info* info) {
  if (!ctx) return IPM_E_ARG;
  if (n_ids < 1 || !ids || max_steps < 0)
    return fail(ctx, IPM_E_ARG, "ipm_step_static: bad arguments");
  for (int k = 0; k < n_ids; ++k)
    if (!get(ctx, ids[k])) return fail(ctx, IPM_E_STATE, "ipm_step_static: unknown problem id");
  std::vector<int> v(ids, ids + n_ids);
  for (size_t a = 0; a < v.size(); ++a)
    for (size_t b = a + 1; b < v.size(); ++b)
      if (v[a] == v[b]) return fail(ctx, IPM_E_ARG, "ipm_step_static: repeated problem id");
  if (!ctx->scratch) return fail(ctx, IPM_E_DEVICE, "ipm_step_static: no static scratch");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (max_steps > 0) {
    bool current = ctx->static_plan && batch_valid(ctx, ctx->static_plan.get(), v);
    if (current) {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      const ScratchSlot& slot = g_scratch[ctx->device];
      current = slot.owner == ctx && slot.tag == ctx->static_plan->scratch_tag;
    }
    if (!current) {
      // plan on the host, then place its arrays in the scratch (no allocation)
      auto B = std::make_unique<BatchPlan>();
      B->owned = false;
      ipm_status st = plan_batch(ctx, v, *B, ctx->static_dps, ctx->static_ups, ctx->static_begins);
      if (st != IPM_OK) return st;
      auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
      const size_t bdp = ctx->static_dps.size() * sizeof(DualParams);
      const size_t bup = ctx->static_ups.size() * sizeof(UpdateParams);
      const size_t bbg = ctx->static_begins.size() * sizeof(int);
      const size_t o_up = up(bdp), o_bg = o_up + up(bup), o_dv = o_bg + up(bbg);
      const size_t total = o_dv + up(bbg);
      if (total > kStaticScratchBytes)
        return fail(ctx, IPM_E_ARG,
                    "ipm_step_static: the launch parameters of these problems need " +
                        std::to_string(total) + " bytes, the static scratch holds " +
                        std::to_string(kStaticScratchBytes));
      unsigned char* base = ctx->scratch;
      B->d_dp = reinterpret_cast<DualParams*>(base);
      B->d_up = reinterpret_cast<UpdateParams*>(base + o_up);
      B->d_begin = reinterpret_cast<int*>(base + o_bg);
      B->d_dev_begin = reinterpret_cast<int*>(base + o_dv);
      // stream-ordered after earlier work on this stream; the wait lets the
      // host copies be reused by the next upload
      if (bdp) HIPCHK(ctx, hipMemcpyAsync(B->d_dp, ctx->static_dps.data(), bdp, hipMemcpyHostToDevice, ctx->stream));
      if (bup) HIPCHK(ctx, hipMemcpyAsync(B->d_up, ctx->static_ups.data(), bup, hipMemcpyHostToDevice, ctx->stream));
      if (bbg) HIPCHK(ctx, hipMemcpyAsync(B->d_begin, ctx->static_begins.data(), bbg, hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ScratchSlot& slot = g_scratch[ctx->device];
        slot.owner = ctx;
        slot.tag = ++g_scratch_uploads;
        B->scratch_tag = slot.tag;
      }
      ctx->static_plan = std::move(B);
    }
    BatchPlan& B = *ctx->static_plan;
    for (int s = 0; s < max_steps; ++s) {
      ipm_status st = launch_batch_step(ctx, B, static_cast<int>(B.steps_done & 1), nullptr);
      if (st != IPM_OK) return st;
      ++B.steps_done;
      for (int id : B.ids) ++get(ctx, id)->step_index;
    }
    for (int k = 0; k < n_ids; ++k) {
      ipm_status st = enqueue_close(ctx, *get(ctx, ids[k]));
      if (st != IPM_OK) return st;
    }
  }
  if (info)
    for (int k = 0; k < n_ids; ++k) {
      ipm_status st = ipm_query(ctx, ids[k], &info[k]);
      if (st != IPM_OK) return st;
    }
  return IPM_OK;
}

ipm_status ipm_query(ipm_ctx* ctx, int id, ipm_step_info* info) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_query: unknown problem id");
  if (!info) return fail(ctx, IPM_E_ARG, "ipm_query: info is NULL");
  StepCtrl hc;
  HIPCHK(ctx, hipMemcpyAsync(&hc, P->d_ctrl, kCtrlHead, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  info->done = (hc.done[hc.steps & 1] || hc.status) ? 1 : 0;
  info->steps = static_cast<long long>(hc.steps);
  info->t = hc.t[hc.steps & 1];
  info->dt = hc.dt_last;
  info->residual = hc.residual;
  info->amax = hc.amax_last;
  info->newton_iters = static_cast<long long>(hc.newton_iters);
  info->cell_updates = static_cast<long long>(hc.steps) * P->cells;
  info->max_iters = static_cast<int>(hc.max_iters);
  info->retard_stage = 0;
  if (P->d_retard) {
    Retard hr;
    HIPCHK(ctx, hipMemcpyAsync(&hr, P->d_retard, sizeof(Retard), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    info->retard_stage = hr.stage;
  }
  const unsigned st = hc.status;
  info->status = st == 0u                  ? IPM_OK
                 : (st & kStNonfinite)     ? IPM_E_NONFINITE
                 : (st & kStRealizability) ? IPM_E_REALIZABILITY
                                           : IPM_E_NEWTON;
  return IPM_OK;
}

ipm_status ipm_moments(ipm_ctx* ctx, int id, double* out, size_t out_len, int out_is_device) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_moments: unknown problem id");
  const size_t cn = static_cast<size_t>(P->cells) * P->M * P->N;
  if (!out || out_len < cn) return fail(ctx, IPM_E_ARG, "ipm_moments: output too small");
  StepCtrl hc;
  HIPCHK(ctx, hipMemcpyAsync(&hc, P->d_ctrl, kCtrlHead, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const double* src = P->d_u[hc.steps & 1];
  HIPCHK(ctx, hipMemcpyAsync(out, src, cn * sizeof(double),
                             out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             ctx->stream));
  if (!out_is_device) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return IPM_OK;
}

ipm_status ipm_dual(ipm_ctx* ctx, int id, double* out, size_t out_len, int out_is_device) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_dual: unknown problem id");
  const size_t cn = static_cast<size_t>(P->cells) * P->M * P->N;
  if (!out || out_len < cn) return fail(ctx, IPM_E_ARG, "ipm_dual: output too small");
  HIPCHK(ctx, hipMemcpyAsync(out, P->d_lam, cn * sizeof(double),
                             out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             ctx->stream));
  if (!out_is_device) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return IPM_OK;
}

ipm_status ipm_cell_degrees(ipm_ctx* ctx, int id, int8_t* out, size_t out_len) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_cell_degrees: unknown problem id");
  if (!out || out_len < static_cast<size_t>(P->cells))
    return fail(ctx, IPM_E_ARG, "ipm_cell_degrees: output too small");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (!P->uneven) {
    std::memset(out, P->degree, static_cast<size_t>(P->cells));
    return IPM_OK;
  }
  StepCtrl hc;
  HIPCHK(ctx, hipMemcpyAsync(&hc, P->d_ctrl, kCtrlHead, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<int8_t> modes(P->cells);
  HIPCHK(ctx, hipMemcpyAsync(modes.data(), P->d_cellN[hc.steps & 1], modes.size(),
                             hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  for (int c = 0; c < P->cells; ++c) {
    int d = 0;
    while (binom_basis(P->p, d) < modes[c]) ++d;
    out[c] = static_cast<int8_t>(d);
  }
  return IPM_OK;
}

ipm_status ipm_problem_sizes(ipm_ctx* ctx, int id, int* m, int* N, int* Q, int* cells) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_problem_sizes: unknown problem id");
  if (m) *m = P->M;
  if (N) *N = P->N;
  if (Q) *Q = P->Q;
  if (cells) *cells = P->cells;
  return IPM_OK;
}

ipm_status ipm_release(ipm_ctx* ctx, int id) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_release: unknown problem id");
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->used -= std::min(ctx->used, P->charged);
  // the cached plan goes stale with the generation (it is never launched
  // again); it stays only so that the next plan can take over its arrays
  ++ctx->gen;
  free_problem(P);
  ctx->problems[id].reset();
  return IPM_OK;
}

ipm_status ipm_serve(ipm_ctx* ctx, int n, ipm_request* reqs, int steps_per_round, int max_active) {
  if (!ctx) return IPM_E_ARG;
  if (n < 0 || (n > 0 && !reqs) || steps_per_round < 1 || max_active < 1)
    return fail(ctx, IPM_E_ARG, "ipm_serve: bad arguments");
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) {
    order[k] = k;
    reqs[k].admitted_s = -1.0;
    reqs[k].finished_s = -1.0;
    reqs[k].steps = 0;
    reqs[k].status = IPM_OK;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  size_t next = 0;
  int finished = 0;
  std::vector<int> active_req, active_id;
  std::vector<CtrlFlags> ctrl;
  // admission, in arrival order, while slots and HBM budget allow
  auto admit = [&]() -> ipm_status {
    while (next < order.size() && reqs[order[next]].arrival_s <= now_s() &&
           static_cast<int>(active_req.size()) < max_active) {
      ipm_request& R = reqs[order[next]];
      int pid = -1;
      ipm_status st = R.problem ? ipm_set_problem(ctx, R.problem, &pid) : IPM_E_ARG;
      if (st == IPM_E_NOMEM && !active_req.empty()) break;  // wait for memory to free up
      ++next;
      if (st != IPM_OK) {
        if (st == IPM_E_DEVICE) return st;
        R.status = st;
        R.finished_s = now_s();
        ++finished;
        continue;
      }
      R.admitted_s = now_s();
      active_req.push_back(order[next - 1]);
      active_id.push_back(pid);
    }
    return IPM_OK;
  };
  while (finished < n) {
    ipm_status st = admit();
    if (st != IPM_OK) return st;
    if (active_req.empty()) {
      if (next < order.size()) {
        const double wait = reqs[order[next]].arrival_s - now_s();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
      }
      continue;
    }
    // one round of batched steps for the problems active now; while it runs,
    // the host prepares the requests that arrived meanwhile (their set-up
    // work queues behind the round on the stream), then the stop flags of
    // the problems the round stepped
    const size_t na = active_id.size();
    st = ipm_step(ctx, static_cast<int>(na), active_id.data(), steps_per_round, nullptr);
    if (st != IPM_OK) return st;
    if ((st = admit()) != IPM_OK) return st;
    ctrl.resize(na);
    if (ctx->poll_cap < na) {
      HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
      if (ctx->d_poll) (void)hipFree(ctx->d_poll);
      if (ctx->h_poll) (void)hipHostFree(ctx->h_poll);
      ctx->d_poll = ctx->h_poll = nullptr;
      ctx->poll_cap = 0;
      const size_t cap = (na + kPollBatch - 1) / kPollBatch * kPollBatch;
      HIPCHK(ctx, hipMalloc(reinterpret_cast<void**>(&ctx->d_poll), cap * sizeof(CtrlFlags)));
      HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->h_poll), cap * sizeof(CtrlFlags)));
      ctx->poll_cap = cap;
    }
    for (size_t k0 = 0; k0 < na; k0 += kPollBatch) {
      PollSources ps{};
      const int nb = static_cast<int>(std::min<size_t>(kPollBatch, na - k0));
      for (int j = 0; j < nb; ++j)
        ps.src[j] = reinterpret_cast<const unsigned long long*>(get(ctx, active_id[k0 + j])->d_ctrl);
      hipLaunchKernelGGL(poll_gather_kernel, dim3(1), dim3(kPollBatch * kFlagWords), 0, ctx->stream,
                         ps, nb, ctx->d_poll + k0 * kFlagWords);
      HIPCHK(ctx, hipGetLastError());
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_poll, ctx->d_poll, na * sizeof(CtrlFlags),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    std::memcpy(ctrl.data(), ctx->h_poll, na * sizeof(CtrlFlags));
    for (size_t k = 0, polled = na; k < polled;) {
      const CtrlFlags& hc = ctrl[k];
      const bool done = hc.done[hc.steps & 1] || hc.status;
      if (!done) {
        ++k;
        continue;
      }
      ipm_request& R = reqs[active_req[k]];
      const int pid = active_id[k];
      ipm_step_info info;
      if ((st = enqueue_close(ctx, *get(ctx, pid))) != IPM_OK) return st;
      if ((st = ipm_query(ctx, pid, &info)) != IPM_OK) return st;
      R.status = info.status;
      R.steps = info.steps;
      if (R.moments_out && info.status == IPM_OK) {
        st = ipm_moments(ctx, pid, R.moments_out, R.moments_len, 0);
        if (st != IPM_OK) R.status = st;
      }
      if ((st = ipm_release(ctx, pid)) != IPM_OK) return st;
      R.finished_s = now_s();
      ++finished;
      active_req.erase(active_req.begin() + static_cast<long>(k));
      active_id.erase(active_id.begin() + static_cast<long>(k));
      ctrl.erase(ctrl.begin() + static_cast<long>(k));
      --polled;
    }
  }
  return IPM_OK;
}

ipm_status ipm_select_degrees(int p, int max_degree, int quad_per_dim, int m, int cells,
                              const double* ic_nodal, double delta_hi, int8_t* out_degree) {
  if (p < 1 || p > 3 || max_degree < 1 || max_degree > 20 || m < 1 || m > 4 || cells < 0 ||
      (cells > 0 && (!ic_nodal || !out_degree)) || !(delta_hi >= 0.0))
    return fail(nullptr, IPM_E_ARG, "ipm_select_degrees: bad arguments");
  if (quad_per_dim < max_degree + 1)
    return fail(nullptr, IPM_E_ARG,
                "ipm_select_degrees: needs quad_per_dim >= max_degree + 1 (exact mode sums)");
  std::vector<double> nodes, w;
  const int Q = tensor_rule(p, quad_per_dim, nodes, w);
  const int N = binom_basis(p, max_degree);
  const std::vector<double> phi = basis_table(p, max_degree, Q, nodes);
  std::vector<int> first(max_degree + 2);  // modes of total degree l: [first[l], first[l+1])
  for (int l = 0; l <= max_degree + 1; ++l) first[l] = l == 0 ? 0 : binom_basis(p, l - 1);
  std::vector<double> uh(N);
  for (int c = 0; c < cells; ++c) {
    // moments of the first conserved variable (Alg. 1 first loop)
    for (int i = 0; i < N; ++i) {
      double a = 0.0;
      for (int q = 0; q < Q; ++q)
        a += w[q] * ic_nodal[(static_cast<size_t>(c) * Q + q) * m] * phi[static_cast<size_t>(q) * N + i];
      uh[i] = a;
    }
    // eq:errorIndicator with an orthonormal basis: <(u_l - u_{l-1})^2> is the
    // sum of squares of the degree-l modes, <u_l^2> that of all modes <= l
    int level = 1;
    double den = uh[0] * uh[0];
    for (int l = 1; l <= max_degree; ++l) {
      double num = 0.0;
      for (int i = first[l]; i < first[l + 1]; ++i) num += uh[i] * uh[i];
      den += num;
      if (l >= 2 && num / den > delta_hi) level = l;
    }
    out_degree[c] = static_cast<int8_t>(level);
  }
  return IPM_OK;
}

ipm_status ipm_autotune(ipm_ctx* ctx, int n_ids, const int* ids, int steps_per_candidate,
                        int* n_tuned) {
  if (!ctx) return IPM_E_ARG;
  if (n_ids <= 0 || !ids || steps_per_candidate <= 0)
    return fail(ctx, IPM_E_ARG, "ipm_autotune: bad arguments");
  for (int k = 0; k < n_ids; ++k)
    if (!get(ctx, ids[k])) return fail(ctx, IPM_E_STATE, "ipm_autotune: unknown problem id");
  if (ctx->timing) return fail(ctx, IPM_E_STATE, "ipm_autotune: kernel timing is on");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  // small-kernel classes by shape
  std::map<std::string, std::vector<std::pair<Problem*, int>>> shapes;
  for (int k = 0; k < n_ids; ++k) {
    Problem* P = get(ctx, ids[k]);
    for (int c = 0; c < kCls; ++c)
      if (P->cls[c].count > 0 && P->cls[c].T == 0 && !P->cls[c].merged)
        shapes[tune_key(*P, P->cls[c])].push_back({P, c});
  }
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  int tuned = 0;
  ipm_status st = IPM_OK;
  for (auto& kv : shapes) {
    const Problem* P0 = kv.second.front().first;
    const DualClass& D0 = P0->cls[kv.second.front().second];
    const int planned = D0.waves;  // D0 is one of the classes the candidates rewrite
    int best = planned;
    // candidates in the order 1 2 4 4 2 1 over consecutive live steps: the
    // work per step drifts as the solution evolves, and the mirrored order
    // gives every candidate the same mean step position, so a linear drift
    // cancels in each candidate's total
    float total[3] = {0.f, 0.f, 0.f};
    bool fits[3] = {false, false, false};
    const int order[6] = {0, 1, 2, 2, 1, 0};
    for (int o = 0; o < 6 && st == IPM_OK; ++o) {
      const int wi = order[o], w = 1 << wi;
      const size_t lds = dual_lds_bytes(P0->M, D0.NP, P0->Q, class_kl(P0->M, P0->kp, D0.NP, 0), w);
      if (lds > ctx->max_lds) continue;
      fits[wi] = true;
      for (auto& pc : kv.second) {
        pc.first->cls[pc.second].waves = w;
        pc.first->cls[pc.second].lds = lds;
      }
      ++ctx->gen;
      if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        st = IPM_E_DEVICE;
        break;
      }
      ctx->batch.reset();
      // one untimed step builds the plan and warms the kernels
      if ((st = ipm_step(ctx, n_ids, ids, 1, nullptr)) != IPM_OK) break;
      if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = IPM_E_DEVICE; break; }
      if ((st = ipm_step(ctx, n_ids, ids, steps_per_candidate, nullptr)) != IPM_OK) break;
      if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = IPM_E_DEVICE;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      total[wi] += ms;
    }
    float best_ms = -1.f;
    for (int wi = 0; wi < 3; ++wi)
      if (fits[wi] && (best_ms < 0.f || total[wi] < best_ms)) {
        best_ms = total[wi];
        best = 1 << wi;
      }
    // the planned shape stays unless another is clearly faster (live steps
    // time with a few per cent of noise)
    const int wd = planned == 1 ? 0 : planned == 2 ? 1 : 2;
    if (fits[wd] && total[wd] <= 1.03f * best_ms) best = planned;
    if (st != IPM_OK) break;
    const size_t lds = dual_lds_bytes(P0->M, D0.NP, P0->Q, class_kl(P0->M, P0->kp, D0.NP, 0), best);
    for (auto& pc : kv.second) {
      pc.first->cls[pc.second].waves = best;
      pc.first->cls[pc.second].lds = lds;
    }
    ctx->tuned_waves[kv.first] = best;
    ++tuned;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ++ctx->gen;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->batch.reset();
  if (st != IPM_OK) return st == IPM_E_DEVICE ? fail(ctx, st, "ipm_autotune: device error") : st;
  if (n_tuned) *n_tuned = tuned;
  return IPM_OK;
}

ipm_status ipm_kernel_timing(ipm_ctx* ctx, int enable, double* dual_ms, double* update_ms,
                             long long* launches) {
  if (!ctx) return IPM_E_ARG;
  if (enable) {
    ctx->timing = true;
    ctx->ev_used = 0;
    ctx->lev_used = 0;
    ctx->lrec.clear();
    return IPM_OK;
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->ltimes.clear();
  for (const auto& r : ctx->lrec) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->lev[r.ev], ctx->lev[r.ev + 1]));
    ipm_launch_time* t = nullptr;
    for (auto& x : ctx->ltimes)
      if (x.m == r.M && x.lanes == r.lanes && x.workgroup == r.workgroup && x.variant == r.variant &&
          x.threads == r.threads)
        t = &x;
    if (!t) {
      ctx->ltimes.push_back(ipm_launch_time{r.M, r.lanes, r.workgroup, r.variant, r.threads, 0, 0.0});
      t = &ctx->ltimes.back();
    }
    ++t->launches;
    t->ms += ms;
  }
  ctx->lrec.clear();
  ctx->lev_used = 0;
  double td = 0.0, tu = 0.0;
  for (size_t k = 0; k + 3 < ctx->ev_used; k += 4) {
    float a = 0.f, b = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&a, ctx->ev[k], ctx->ev[k + 1]));
    HIPCHK(ctx, hipEventElapsedTime(&b, ctx->ev[k + 2], ctx->ev[k + 3]));
    td += a;
    tu += b;
  }
  if (dual_ms) *dual_ms = td;
  if (update_ms) *update_ms = tu;
  if (launches) *launches = static_cast<long long>(ctx->ev_used / 4);
  ctx->timing = false;
  ctx->ev_used = 0;
  return IPM_OK;
}

ipm_status ipm_launch_times(ipm_ctx* ctx, ipm_launch_time* out, int cap, int* n) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return fail(ctx, IPM_E_ARG, "ipm_launch_times: bad arguments");
  *n = static_cast<int>(ctx->ltimes.size());
  for (int k = 0; k < *n && k < cap; ++k) out[k] = ctx->ltimes[k];
  return IPM_OK;
}

ipm_status ipm_class_stats(ipm_ctx* ctx, int id, ipm_class_stat* out, int cap, int* n) {
  Problem* P = get(ctx, id);
  if (!P) return fail(ctx, IPM_E_STATE, "ipm_class_stats: unknown problem id");
  if (!n || cap < 0 || (cap > 0 && !out)) return fail(ctx, IPM_E_ARG, "ipm_class_stats: bad arguments");
  std::vector<unsigned long long> blk(static_cast<size_t>(P->dual_blocks) * kBlkStats);
  HIPCHK(ctx, hipMemcpyAsync(blk.data(), P->d_blk, blk.size() * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  int k = 0;
  for (int c = 0; c < kCls; ++c) {
    const DualClass& D = P->cls[c];
    if (!D.configured || D.n_max == 0) continue;
    ipm_class_stat s{};
    s.size_class = c;
    s.workgroup = D.T > 0 ? 1 : 0;
    s.lanes = D.NP;
    s.variant = reg_variant(D.prec, D.T, D.NP, P->Q);
    s.n_min = D.n_min;
    s.n_max = D.n_max;
    s.cells = D.count;
    for (int b = D.blk_off; b < D.blk_off + D.blk_cnt; ++b) {
      s.iterations += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b)]);
      s.listed += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b) + 2]);
      s.fresh += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b) + 3]);
    }
    if (k < cap) out[k] = s;
    ++k;
    if (D.chord) {  // the chord kernel's counters (variant 10)
      ipm_class_stat t = s;
      t.variant = 10;
      t.listed = t.iterations = t.fresh = 0;
      for (int b = D.cblk_off; b < D.cblk_off + D.cblk_cnt; ++b) {
        t.iterations += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b)]);
        t.listed += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b) + 2]);
        t.evaluations += static_cast<long long>(blk[kBlkStats * static_cast<size_t>(b) + 3]);
      }
      if (k < cap) out[k] = t;
      ++k;
    }
  }
  *n = k;
  return IPM_OK;
}

}  // extern "C"
