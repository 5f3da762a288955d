/*
 * ipm.h -- C ABI of libipm, an MI355X (gfx950) implementation of the hot
 * path of the Intrusive Polynomial Moment (IPM) method for hyperbolic
 * conservation laws with uncertain initial data (Kusch, Wolters, Frank,
 * arXiv:1912.09238).
 *
 * One call to ipm_step advances each listed problem by up to max_steps time
 * steps.  A time step is, for every cell j,
 *   1. the dual solve lambda_j = argmin L(lambda; uhat_j) of eq:L by Newton
 *      iterations lambda <- d(lambda, uhat_j) (eq:dualIterationFunction)
 *      until eq:tauCrit holds (Alg. 1), or exactly one Newton step in the
 *      one-shot mode (eq:oneshotIPM, Alg. 2);
 *   2. the kinetic numerical flux of the ansatz u_s(lambda^T phi) at the
 *      quadrature nodes and the moment update c(lambda_l, lambda_c,
 *      lambda_r) of eq:momentIterationFunction in the quadrature form
 *      eq:momentUpQuadrature (Sec. 3.1 and Sec. 6);
 * with the time step dt = CFL dx / a_max taken from the largest wave speed
 * of the current ansatz over all cells and nodes (2D: CFL / (a_x/dx +
 * a_y/dy)), the last step clipped to t_end.  Every step runs in HIP kernels
 * on the device; the host only enqueues.
 *
 * Conventions
 *  - Every call returns an ipm_status; the message of the last failure is
 *    ipm_last_error(ctx).
 *  - Host input arrays are read and copied during the call; the caller keeps
 *    ownership.  Device state is owned by the context.
 *  - Moment and dual arrays use the layout [cell][m][N]: cell-major, then
 *    the m conserved variables, then the N basis functions in graded order
 *    (total degree ascending, first exponent descending; phi_0 = 1 first).
 *    Cells are numbered c = iy * nx + ix.  Nodal arrays are [cell][Q][m]
 *    with the tensor Gauss-Legendre nodes in the order ipm_quadrature gives.
 *  - ipm_step is asynchronous on the context's stream unless info != NULL.
 *  - A numerical failure of a problem (Newton not converged, ansatz outside
 *    the entropy's domain, non-finite values) is sticky for that problem and
 *    stops it; other problems go on.
 *  - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef IPM_H
#define IPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipm_ctx ipm_ctx;

typedef enum {
  IPM_OK = 0,
  IPM_E_ARG = -1,           /* invalid argument (message names it) */
  IPM_E_STATE = -2,         /* unknown problem id or call out of order */
  IPM_E_NOMEM = -3,         /* device memory or admission budget exhausted */
  IPM_E_REALIZABILITY = -4, /* ansatz outside the closure's domain */
  IPM_E_NEWTON = -5,        /* dual not converged within max_newton */
  IPM_E_NONFINITE = -6,     /* NaN/Inf in the state */
  IPM_E_DEVICE = -7,        /* HIP runtime error */
  IPM_E_BUSY = -8           /* no free problem slot */
} ipm_status;

enum { IPM_BURGERS_1D = 0, IPM_EULER_1D = 1, IPM_EULER_2D = 2 };
/* entropies (Sec. 2 eq:primalProblem): quadratic |u|^2/2 gives stochastic
   Galerkin; log-barrier (u-u_-)ln(u-u_-)+(u_+-u)ln(u_+-u) for scalar
   problems; the Euler entropy -rho ln(rho^-gamma (E-|m|^2/(2 rho))) of App. B */
enum { IPM_ENT_QUADRATIC = 0, IPM_ENT_LOG_BARRIER = 1, IPM_ENT_EULER = 2 };
/* With the quadratic entropy the Euler equations' ansatz is the SG
   expansion; a node with non-positive density or pressure is reported as
   IPM_E_REALIZABILITY (the failure of stochastic Galerkin, Sec. 7). */
/* deterministic numerical flux g of the kinetic flux eq:numericalFluxIPM;
   IPM_FLUX_SG_ANALYTIC: the Lax-Friedrichs flux of the stochastic-Galerkin
   moment system of Burgers' equation with the triple products
   <phi_a phi_b phi_i> (App. A, eq:numFluxAnalytic), O(N^3) per face instead
   of O(N Q); Burgers with the quadratic entropy, outflow or periodic
   boundaries, fixed degrees, N <= 16.  It equals the LF kinetic flux when
   the rule integrates degree 3M exactly. */
enum { IPM_FLUX_LF = 0, IPM_FLUX_RUSANOV = 1, IPM_FLUX_SG_ANALYTIC = 2 };
enum { IPM_BC_OUTFLOW = 0, IPM_BC_PERIODIC = 1, IPM_BC_DIRICHLET = 2 };
/* arithmetic of the Hessian assembly (the Newton update, the SPD solve --
   Gauss-Jordan elimination without pivoting, n^3 flops against Cholesky's
   n^3/3, chosen for its broadcast-only data flow on register rows --, the
   gradient and the tau test are always FP64).  IPM_PREC_BF16: split-BF16 products on
   the matrix cores for cells of 65..96 unknowns; smaller cells (register-row
   kernels) and larger ones (whose FP32 block area would cost occupancy)
   keep the FP64 assembly.  IPM_PREC_FP32 is rejected (no faster than FP64
   here). */
enum { IPM_PREC_FP64 = 0, IPM_PREC_FP32 = 1, IPM_PREC_BF16 = 2 };
/* quadrature rule for xi ~ U(-1,1)^p (Sec. 3.1 <.>_Q; Sec. 7 compares
   tensorized and sparse Clenshaw-Curtis grids): tensor Gauss-Legendre or
   tensor Clenshaw-Curtis with quad_per_dim points per dimension, or the
   Smolyak sparse grid of nested Clenshaw-Curtis rules (1, 3, 5, 9, ...
   points) of level quad_per_dim (0..11; p = 3: 1, 7, 25, 69, 177, 441, ...
   nodes).  Sparse grids carry negative weights, so the dual Hessian can
   lose definiteness (the failure Sec. 7 reports from order 3 on). */
enum { IPM_QUAD_GAUSS_LEGENDRE = 0, IPM_QUAD_CLENSHAW_CURTIS = 1, IPM_QUAD_CC_SPARSE = 2 };

typedef struct {
  int device;               /* HIP device ordinal */
  void *hip_stream;         /* hipStream_t to order all work on; NULL: the null stream */
  size_t hbm_budget_bytes;  /* admission limit for all problems (0: no limit) */
  int max_problems;         /* problem slots (0: 1024) */
} ipm_config;

typedef struct {
  int equation;             /* IPM_BURGERS_1D | IPM_EULER_1D | IPM_EULER_2D */
  int entropy;              /* IPM_ENT_* (Burgers: quadratic or log-barrier; Euler: quadratic or Euler) */
  int flux;                 /* IPM_FLUX_* */
  double gamma;             /* ratio of specific heats (Euler), > 1 */
  double u_minus, u_plus;   /* log-barrier bounds, u_minus < u_plus */
  int p;                    /* uncertain dimensions, 1..3; xi ~ U(-1,1)^p */
  int degree;               /* total degree M; N = binomial(M+p, p) (eq:numberBasisFcts) */
  const int8_t *cell_degree;/* optional [cells] per-cell total degree in 0..degree (NULL: uniform) */
  int quad_per_dim;         /* tensor Gauss-Legendre points per dimension; Q = quad_per_dim^p */
  double cfl;               /* dt = cfl * dx / a_max */
  double t_end;             /* stop time (> 0), or 0 for no time limit */
  double tau;               /* dual tolerance of eq:tauCrit (absolute) */
  double steady_eps;        /* stop when eq:residualSteady <= steady_eps (0: never) */
  int max_newton;           /* Newton iterations per cell and step before IPM_E_NEWTON */
  int one_shot;             /* 1: one Newton step per time step (Alg. 2) */
  int precision;            /* IPM_PREC_* */
  int nx, ny;               /* cells per direction (ny = 1 in 1D) */
  double x0, x1, y0, y1;    /* domain */
  int bc[4];                /* x-, x+, y-, y+ (periodic must be paired) */
  const double *ic_nodal;   /* [cells][Q][m] u_IC at cell centres and nodes, or NULL */
  const double *ic_moments; /* [cells][m][N] initial moments (used if ic_nodal == NULL) */
  const double *ic_dual;    /* optional [cells][m][N] warm start of the dual (resume) */
  const double *dirichlet;  /* [4][Q][m] nodal ghost states of Dirichlet sides, or NULL */
  /* Dynamic adaptivity (Sec. 5, Alg. ad-IPM).  adapt = 1: after its dual
     solve every cell takes the smoothness indicator eq:errorIndicator of the
     first conserved variable of its ansatz at its current level (levels are
     total degrees); below delta_lo it moves one level down, above delta_hi
     one level up, within [min_degree, degree].  The moment update projects
     on the new level (eq:adaptiveFVUpdate) and the dual keeps the modes of
     the new level (zero-padded when it rises).  The levels start at
     cell_degree (NULL: degree).  Needs min_degree >= 1, delta_lo <= delta_hi
     and quad_per_dim >= degree + 1 (the indicator's averages are then exact
     sums of squared modes).  With one_shot = 1 this is the adaptive one-shot
     of Alg. adosIPM (one Newton step per cell and pseudo-time step).
     adapt = 0: the per-cell degrees stay fixed and these fields are ignored. */
  int adapt;
  int min_degree;
  double delta_lo, delta_hi;
  /* Refinement retardation (Sec. 5, Alg. adosIPM), for adapt = 1 and
     steady_eps > 0: stage l caps every level at retard_degree[l] (a cell
     takes the smaller of the indicator's level and the cap); the stage
     advances when the steady residual eq:residualSteady of a step falls to
     retard_eps[l]; the steady stop applies only in the last stage (whose
     tolerance is unused).  1..16 stages, degrees non-decreasing within
     [min_degree, degree]; the arrays are copied.  n_retard = 0: no cap. */
  int n_retard;
  const int *retard_degree;
  const double *retard_eps;
  int quad_rule;            /* IPM_QUAD_*; 0 (Gauss-Legendre) for the fields above */
  /* Inexact-Hessian Newton (the outlook of Sec. 7: do not recompute the
     Hessian at every iteration) for the cells on the workgroup kernel (more
     than 64 unknowns, or many quadrature nodes): 1 = each such cell keeps
     the inverse of its last freshly assembled Hessian in device memory
     (rounded to FP32, NP x NP floats with NP = n rounded up to 8, 16, 32 or
     64 for n <= 64 and to a multiple of 16 above: 4 KB per cell at n = 30,
     about 37 KB at n = 84) and takes later
     Newton steps, in this and following time steps, as d = H_old^-1 grad L
     (on fixed degrees with the L-BFGS correction of the cell's last accepted
     step of the same time step) while each such step contracts the dual
     residual by reuse_theta;
     otherwise the inverse is retired and the next iteration (one-shot: of
     the next pseudo-time step) assembles and inverts afresh.  The tau test is
     unchanged, so the dual still converges to tau; results agree with exact
     Newton within the dual tolerance, not bit for bit.  With adaptive
     levels each cell keeps one slot of the largest class's size and a level
     change retires the cell's inverse.
     2 = the same for every cell, also on the register-row kernels (n <= 64;
     slower than exact Newton on the 1D workloads measured, where those
     solves are cheap and the launches latency bound; with it the Newton
     launches of a problem's size classes stay separate).  0 = exact Newton. */
  int hessian_reuse;
  /* Inexact-Hessian Newton: a step from the stored inverse is kept only if it
     reduces the dual residual to at most reuse_theta times its value before
     the step; 0 selects 0.5.  In [0, 1). */
  double reuse_theta;
} ipm_problem;

typedef struct {
  int status;               /* ipm_status of the problem (sticky) */
  int done;                 /* reached t_end or steady_eps, or failed */
  long long steps;          /* completed time steps */
  double t, dt;             /* time reached, last time step */
  double residual;          /* last eq:residualSteady value */
  double amax;              /* last largest wave speed */
  long long newton_iters;   /* Newton updates summed over cells and steps */
  long long cell_updates;   /* cells x completed steps */
  int max_iters;            /* largest Newton count of one cell in one step */
  int retard_stage;         /* current refinement-retardation stage (0 if none) */
} ipm_step_info;

/* One request of the serving loop (ipm_serve). */
typedef struct {
  const ipm_problem *problem; /* the solve; inputs must stay valid until it is admitted */
  double arrival_s;         /* arrival, seconds after ipm_serve starts */
  double *moments_out;      /* host [cells][m][N], written when it finishes (nullable) */
  size_t moments_len;       /* capacity of moments_out in doubles */
  /* filled by ipm_serve: */
  double admitted_s;        /* when its state was set up on the device (-1: never) */
  double finished_s;        /* when its moments were back on the host */
  long long steps;          /* completed time steps */
  int status;               /* ipm_status of the request */
  int reserved;
} ipm_request;

/* Create a context on cfg->device.  *out receives the handle. */
ipm_status ipm_create(const ipm_config *cfg, ipm_ctx **out);

/* Release every problem and the context. */
ipm_status ipm_destroy(ipm_ctx *ctx);

/* Tensor Gauss-Legendre rule for xi ~ U(-1,1)^p (Sec. 3.1 quadrature
   <h>_Q with the density folded into the weights, so sum(weights) = 1):
   nodes [Q][p] with the first coordinate varying slowest.  cap = capacity of
   weights in entries; returns IPM_E_ARG if Q > cap.  Host only, no device. */
ipm_status ipm_quadrature(int p, int quad_per_dim, double *nodes, double *weights, int cap);

/* Number of nodes of a quadrature rule (IPM_QUAD_*, param = points per
   dimension or sparse level), 0 for invalid arguments.  Host only. */
int ipm_quadrature_size(int rule, int p, int param);

/* Nodes [Q][p] and weights [Q] (sum 1) of a rule, as problems with that
   quad_rule use them; cap = capacity of weights.  Tensor rules order nodes
   with the first coordinate slowest; sparse grids in ascending order of the
   nodes' indices on the finest Clenshaw-Curtis grid.  Host only. */
ipm_status ipm_quadrature_rule(int rule, int p, int param, double *nodes, double *weights, int cap);

/* Number of basis functions N = binomial(degree + p, p). */
int ipm_basis_size(int p, int degree);

/* Basis table Phi [Q][N], Phi[q][i] = phi_i(xi_q), of the orthonormal
   total-degree Legendre basis (Sec. 2, gPC basis; App. A table A) at the
   nodes of ipm_quadrature, as the library uploads it.  cap = capacity of Phi
   in entries.  Host only, no device. */
ipm_status ipm_basis_table(int p, int degree, int quad_per_dim, double *Phi, int cap);

/* Copy a problem to the device: tables, IC projection (Alg. 1 first loop),
   initial dual from the entropy variables, converged to tau.  Synchronous.
   IPM_E_NOMEM when the problem does not fit the HBM budget (admission). */
ipm_status ipm_set_problem(ipm_ctx *ctx, const ipm_problem *pb, int *problem_id);

/* Enqueue up to max_steps time steps (Alg. 1 time loop; Alg. 2 pseudo-time
   loop for one-shot problems) for each of the n_ids problems.  Steps after a
   problem is done are skipped on the device.  With two or more distinct ids
   the problems advance together: each step is one batched Newton launch per
   kernel shape (all problems' cells of that shape) and one batched update
   launch per shape, replayed from two device graphs (one per step parity)
   that are built on the first call for this id list and reused while the
   list and the problems' step counts match.  A single problem whose cells
   span several Newton kernel shapes (per-cell or adaptive degrees) steps the
   same way, so that its Newton launches overlap.  The results are those of
   stepping each problem alone.  ids must be distinct (IPM_E_ARG).  If info is
   not NULL the call waits and fills info[k] for ids[k]. */
ipm_status ipm_step(ipm_ctx *ctx, int n_ids, const int *ids, int max_steps,
                    ipm_step_info *info);

/* ipm_step for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): the
   same batched launches as ipm_step with two or more ids (one problem is
   also allowed), launched one by one on the context's stream without a
   graph, and the results equal ipm_step's bit for bit.  The launches'
   parameter arrays and block offsets live in a fixed device array of
   512 KiB per GPU (defined in the library, held until the process ends),
   not in allocations of the call; ids whose arrays would exceed it (per
   problem and step parity 272 bytes per Newton launch -- one per size
   class, two for a class with a chord kernel -- plus 384 for the update and
   8 bytes of block offsets per launch: about 5.3 KB over both parities for
   a problem with four chord classes, so about 99 such problems) fail with
   IPM_E_ARG and a message naming the size.  The problems' own state comes from ipm_set_problem as for
   ipm_step.  Every call on a GPU shares that GPU's array, which keeps the
   last call's contents: the first call for an id list (or after another
   list, context or ipm_step has used the array or moved the problems)
   uploads the arrays and waits for the stream once; later calls with the
   same list launch at once.  Calls that overlap on one GPU (two contexts or
   threads at the same time) race on the array and are not allowed.  Errors
   as ipm_step; info as ipm_step (the call waits when info != NULL). */
ipm_status ipm_step_static(ipm_ctx *ctx, int n_ids, const int *ids, int max_steps,
                           ipm_step_info *info);

/* Static per-cell total degree for the batching form (Sec. 5: the first
   entry of the smoothness indicator eq:errorIndicator, computed from the
   first conserved variable's moments at t = 0).  Levels are total degrees
   1..max_degree; a cell gets the highest level l >= 2 whose indicator
   S_l = <(u_l - u_{l-1})^2> / <u_l^2> exceeds delta_hi, else 1 (a static
   reading of the raise rule, with the thresholds ordered as delta_lo <
   delta_hi).  ic_nodal: host [cells][Q][m] values u_IC(x_j, xi_q) on the
   tensor rule of quad_per_dim points (quad_per_dim >= max_degree + 1, so
   that the averages are exact sums of squared modes).  out_degree: host
   [cells].  Needs no context and no device; errors: IPM_E_ARG. */
ipm_status ipm_select_degrees(int p, int max_degree, int quad_per_dim, int m, int cells,
                              const double *ic_nodal, double delta_hi, int8_t *out_degree);

/* Serving loop (a runtime around the method; no passage of the paper).  Runs
   the n requests against the wall clock: a request is admitted once it has
   arrived, fewer than max_active requests are on the device and its state
   fits the context's HBM budget (ipm_set_problem's IPM_E_NOMEM is the
   admission signal; a request that cannot fit even alone fails with it).
   Admitted requests keep their moment and dual state resident and advance
   together, steps_per_round batched time steps per round (ipm_step with all
   active ids); requests that arrive while a round runs are set up meanwhile
   (their set-up work queues behind the round on the context's stream) and
   join the next round; finished ones leave at round boundaries (moments
   copied to moments_out, state released).  The stop flags of the active
   problems come back in one copy per round.  Every request's result
   equals that of stepping it alone.  Blocks until every request finished or
   failed; per-request failures are reported in reqs[k].status, the return
   value only reports device or argument errors. */
ipm_status ipm_serve(ipm_ctx *ctx, int n, ipm_request *reqs, int steps_per_round, int max_active);

/* Autotuner of the batched launches (no passage of the paper: a launch-shape
   choice).  For every small-cell Newton kernel shape among the problems, runs
   1 + steps_per_candidate real time steps of all n_ids problems with 1, 2,
   4, 4, 2 and 1 wavefronts per block (mirrored, so that the drift of the work
   per step cancels), keeps the shape of the smallest total time (the planned
   shape unless another is more than 3 % faster) and remembers it for
   problems of the same shape created later in this context.  The choice does not change
   any result (each cell's arithmetic is independent of the block shape); the
   timed steps advance the problems.  *n_tuned (nullable) = shapes tuned. */
ipm_status ipm_autotune(ipm_ctx *ctx, int n_ids, const int *ids, int steps_per_candidate,
                        int *n_tuned);

/* Wait for the context's stream and fill *info for one problem. */
ipm_status ipm_query(ipm_ctx *ctx, int id, ipm_step_info *info);

/* Current moments [cells][m][N] of a problem: the stochastic-Galerkin moments
   uhat_i = <u phi_i> of the state on the gPC basis (Sec. 2, the moment
   system that eq:momentIterationFunction advances); modes above a cell's
   degree are zero.  out_is_device: out is a device pointer (copy ordered on the
   context stream, asynchronous) or a host pointer (synchronous).
   out_len = capacity of out in doubles. */
ipm_status ipm_moments(ipm_ctx *ctx, int id, double *out, size_t out_len, int out_is_device);

/* Current dual state [cells][m][N] (checkpoint; pass back as ic_dual). */
ipm_status ipm_dual(ipm_ctx *ctx, int id, double *out, size_t out_len, int out_is_device);

/* Current total degree (refinement level) of every cell of a problem:
   host out [cells], capacity out_len.  Waits for the context's stream.  For
   a problem with fixed degrees these are the degrees it was created with. */
ipm_status ipm_cell_degrees(ipm_ctx *ctx, int id, int8_t *out, size_t out_len);

/* Sizes of a problem: conserved variables, basis functions, nodes, cells. */
ipm_status ipm_problem_sizes(ipm_ctx *ctx, int id, int *m, int *N, int *Q, int *cells);

/* Bytes of device memory a problem would take (admission estimate). */
size_t ipm_problem_footprint(const ipm_problem *pb);

/* Free a problem's slot and device memory. */
ipm_status ipm_release(ipm_ctx *ctx, int id);

/* Kernel timing with HIP events on the context's stream.  enable = 1 clears
   the record and brackets every following dual-solve and update launch with
   its own event pair; enable = 0 waits for the stream, returns the summed
   device time of the dual-solve and of the update kernels in milliseconds
   and the number of steps recorded, and stops recording. */
ipm_status ipm_kernel_timing(ipm_ctx *ctx, int enable, double *dual_ms, double *update_ms,
                             long long *launches);

/* Device time of the batched Newton launches of the last timing window
   (ipm_kernel_timing enable = 1 ... enable = 0; batched ipm_step only, which
   then launches one kernel at a time): per kernel shape, the launches and
   their summed milliseconds.  Measurement helper, no passage of the paper. */
typedef struct {
  int m;          /* conserved variables of the kernel */
  int lanes;      /* register-row kernel: lanes per cell; workgroup kernel: 16 T rows */
  int workgroup;  /* 1: one workgroup per cell (T x T register tiles), 0: register rows */
  int variant;    /* bit 0: BF16 MFMA Hessian; bit 1: stored inverse Hessians;
                     bit 2: register rows holding all nodes at once (Q <= lanes) */
  int threads;    /* threads per block */
  long long launches;
  double ms;
} ipm_launch_time;
ipm_status ipm_launch_times(ipm_ctx *ctx, ipm_launch_time *out, int cap, int *n);

/* Newton counters of a problem per size class (cumulative since set-up;
   waits for the context's stream): the kernel shape of the class's launches,
   the range of unknowns n = m N of the cells they solve, the class's cells,
   and how many cells the launches solved (listed), their Newton iterations
   (eq:dualIterationFunction steps) and how many of these assembled a fresh
   Hessian (the rest reused a stored inverse).  Classes with a chord kernel
   (inexact-Hessian Newton on fixed degrees) report it as a second entry
   with variant 10, whose evaluations counts its passes over the quadrature
   nodes (the ansatz and gradient at the entry point and at every line-search
   trial; 0 in the other entries).  *n = classes reported (at most cap are
   written).  Measurement helper. */
typedef struct {
  int size_class;
  int workgroup;  /* as in ipm_launch_time */
  int lanes;
  int variant;
  int n_min, n_max;
  long long cells;
  long long listed;
  long long iterations;
  long long fresh;
  long long evaluations;
} ipm_class_stat;
ipm_status ipm_class_stats(ipm_ctx *ctx, int id, ipm_class_stat *out, int cap, int *n);

/* Message of the last failing call on ctx (owned by ctx, valid until the
   next call).  ctx may be NULL for errors of ipm_create. */
const char *ipm_last_error(const ipm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
