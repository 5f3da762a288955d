/*
 * ipm_oracle.h -- plain FP64 CPU oracle of the Intrusive Polynomial Moment
 * (IPM) hot path of Kusch, Wolters and Frank, "Intrusive acceleration
 * strategies for uncertainty quantification for hyperbolic systems of
 * conservation laws" (arXiv:1912.09238).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  The
 * product library never links, includes or calls it, and the two share no
 * code (tables, closures, solvers and the scheme are written twice).
 *
 * Everything is FP64, scalar loops, one cell at a time.  OpenMP is used only
 * to run independent cells of one step on several cores; per-cell results
 * do not depend on the thread count.
 *
 * Parity pins: every function here is pinned by the "not gpu" tests against
 * closed forms, special cases (stochastic Galerkin, deterministic finite
 * volumes, coupled collocation at N = Q), invariants (conservation, maximum
 * principle, dual round trip, decay of the total entropy) and brute-force
 * collocation.  The exact moment trajectories for N < Q with a
 * non-quadratic entropy are pinned by the entropy decay only, not to exact
 * values ("parity unpinned" for their exact values).
 */
#ifndef IPM_ORACLE_H
#define IPM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXM 4
#define ORC_MAX_RETARD 16

enum { ORC_BURGERS_1D = 0, ORC_EULER_1D = 1, ORC_EULER_2D = 2 };
enum { ORC_ENT_QUADRATIC = 0, ORC_ENT_LOG_BARRIER = 1, ORC_ENT_EULER = 2 };
/* ORC_FLUX_SG_ANALYTIC: App. A, eq:numFluxAnalytic -- the Lax-Friedrichs flux
   of the stochastic-Galerkin moment system of Burgers' equation with the
   triple products <phi_n phi_k phi_i>, applied to the duals (quadratic
   entropy: the dual is the SG moment vector); 1D Burgers only */
enum { ORC_FLUX_LF = 0, ORC_FLUX_RUSANOV = 1, ORC_FLUX_SG_ANALYTIC = 2 };
enum { ORC_BC_OUTFLOW = 0, ORC_BC_PERIODIC = 1, ORC_BC_DIRICHLET = 2 };
/* quadrature for xi ~ U(-1,1)^p: tensor Gauss-Legendre, tensor
   Clenshaw-Curtis (points per dimension), Clenshaw-Curtis sparse grid
   (Smolyak, nested 1, 3, 5, 9, ... point rules; the parameter is the level) */
enum { ORC_QUAD_GL = 0, ORC_QUAD_CC = 1, ORC_QUAD_CC_SPARSE = 2 };

/* status bits, sticky per problem */
enum {
  ORC_ST_NEWTON = 1,        /* dual not converged within max_newton */
  ORC_ST_REALIZABILITY = 2, /* ansatz outside the closure's domain */
  ORC_ST_NONFINITE = 4,     /* NaN/Inf in gradient, wave speed or moments */
  ORC_ST_CHOLESKY = 8,      /* non-positive pivot in the Hessian factor */
  ORC_ST_LINESEARCH = 16    /* no admissible step after 60 halvings */
};

typedef struct {
  int equation;          /* ORC_BURGERS_1D | ORC_EULER_1D | ORC_EULER_2D */
  int entropy;           /* ORC_ENT_* */
  int flux;              /* ORC_FLUX_* */
  double gamma;          /* ratio of specific heats (Euler) */
  double u_minus, u_plus;/* log-barrier bounds (Burgers) */
  int p;                 /* number of uncertain dimensions */
  int degree;            /* total degree M of the basis */
  int quad_per_dim;      /* tensor Gauss-Legendre points per dimension */
  int nx, ny;            /* cells (ny = 1 in 1D) */
  double x0, x1, y0, y1; /* domain */
  int bc[4];             /* x-, x+, y-, y+ : ORC_BC_* */
  double cfl, t_end, tau, steady_eps;
  int max_newton, one_shot;
  /* dynamic adaptivity (Sec. 5, Alg. ad-IPM): after each dual solve a cell
     moves one level (total degree) down when the indicator of its ansatz at
     its level is below delta_lo, one up when it is above delta_hi, within
     [min_degree, degree]; the moment update projects on the new level and
     the dual drops the modes above it.  adapt = 0: levels stay fixed. */
  int adapt, min_degree;
  double delta_lo, delta_hi;
  /* refinement retardation (Sec. 5, Alg. adosIPM), steady runs with
     adaptivity: stage l caps every level at retard_degree[l]; the stage
     advances when the steady residual falls to retard_eps[l]; the run stops
     at steady_eps only in the last stage.  n_retard = 0: no cap. */
  int n_retard;
  int retard_degree[ORC_MAX_RETARD];
  double retard_eps[ORC_MAX_RETARD];
  int quad_rule;         /* ORC_QUAD_*; quad_per_dim is the sparse level for ORC_QUAD_CC_SPARSE */
} orc_problem;

typedef struct {
  double t, dt, residual, amax;
  long long steps, newton_iters, cell_updates;
  int max_iters, status, done;
  int retard_stage;      /* current stage of the refinement retardation */
} orc_info;

typedef struct orc_state orc_state;

/* tables */
int orc_num_basis(int p, int degree);
int orc_gauss_legendre(int n, double *x, double *w);
int orc_quadrature(int p, int qpd, double *nodes /*[Q][p]*/, double *w /*[Q], sum 1*/);
int orc_multi_indices(int p, int degree, int *idx /*[N][p]*/);
int orc_clenshaw_curtis(int n, double *x, double *w /*sum 2*/);
int orc_quadrature_size(int rule, int p, int param);
int orc_quadrature_rule(int rule, int p, int param, double *nodes /*[Q][p]*/, double *w /*sum 1*/);
void orc_basis_eval(int p, int degree, int Q, const double *nodes, double *Phi /*[Q][N]*/);

/* Smoothness indicator of Sec. 5 (eq:errorIndicator) for one scalar field
   given at the Q nodes: moments up to total degree L by quadrature, then for
   levels l = 1..L (level l = total degree l)
     S[l-1] = <(u_l - u_{l-1})^2>_Q / <u_l^2>_Q,  u_l = sum_{|i|<=l} u_i phi_i,
   with every average taken by the quadrature rule. */
void orc_indicator(int p, int L, int qpd, const double *u_nodes /*[Q]*/, double *S /*[L]*/);

/* Static per-cell level at t = 0 (first entry of the indicator: the first
   conserved variable): the highest level l >= 2 with S_l > delta_hi, else 1.
   ic_nodal [cells][Q][m]; out [cells] total degree in 1..L. */
void orc_select_degrees(int p, int L, int qpd, int m, int cells, const double *ic_nodal,
                        double delta_hi, signed char *out);

/* closures at one node; m = 1 (scalar) or d+2 (Euler) */
int orc_closure(int entropy, int m, double gamma, double um, double up,
                const double *Lam, double *u, double *J /*[m][m]*/, double *sstar);
int orc_entropy_grad(int entropy, int m, double gamma, double um, double up,
                     const double *u, double *Lam);
double orc_entropy(int entropy, int m, double gamma, double um, double up, const double *u);

/* problem state */
orc_state *orc_create(const orc_problem *pb, const signed char *cell_degree,
                      const double *ic_nodal /*[cells][Q][m]*/,
                      const double *dirichlet_nodal /*[4][Q][m] or NULL*/);
void orc_destroy(orc_state *S);
void orc_sizes(const orc_state *S, int *m, int *N, int *Q, int *cells);
int orc_step(orc_state *S, int max_steps, orc_info *info);
void orc_get_info(const orc_state *S, orc_info *info);
void orc_get_moments(const orc_state *S, double *out /*[cells][m][N]*/);
void orc_set_moments(orc_state *S, const double *in);
void orc_get_dual(const orc_state *S, double *out /*[cells][m][N]*/);
void orc_set_dual(orc_state *S, const double *in);
void orc_get_iters(const orc_state *S, int *out /*[cells]*/);
void orc_get_degrees(const orc_state *S, signed char *out /*[cells] current total degree*/);
int orc_get_nodal(const orc_state *S, double *out /*[cells][Q][m]*/);
void orc_tables(const orc_state *S, double *nodes, double *w, double *Phi);

/* one cell's dual problem (full degree of the problem) */
int orc_dual_cost(const orc_state *S, const double *lam, const double *uhat,
                  double *L, double *grad /*[m][N]*/, double *H /*[mN][mN]*/);
int orc_dual_solve(const orc_state *S, const double *uhat, double *lam, int one_shot, int *iters);
int orc_moments_of_dual(const orc_state *S, const double *lam, double *uhat);

int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
