/*
 * ipm_oracle.c -- plain FP64 CPU oracle of the IPM hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see ipm_oracle.h).  Written from the paper's
 * equations; citations name the section / equation / algorithm followed.
 *
 * Readings where the paper is silent or garbled (each one also listed in
 * the design notes of the repository):
 *   - E-derivative of the Euler entropy gradient: the printed form is a
 *     garbled reciprocal; the consistent value is -rho/eps (App. B).
 *   - The exponent of alpha(Lambda) in App. B carries -2*Lambda_4*gamma; the
 *     inverse of the printed gradient needs +2*Lambda_4*gamma.  Moments do
 *     not depend on this shift (phi_0 = 1 absorbs it).
 *   - tau test (eq:tauCrit): sum over the m conserved variables of the
 *     Euclidean norm over the N modes, absolute.
 *   - Newton globalization (Sec. 3.1 only says "Newton's method"): if the
 *     dual residual exceeds 1e-6, backtrack t <- t/2 until the Armijo
 *     condition L(l - t d) <= L(l) - 1e-4 t g.d holds (inadmissible = +inf);
 *     otherwise t = 1.  One-shot always takes t = 1 (Alg. 2).
 *   - Moment update uses h(lambda_c) as the old-moment term, as in
 *     eq:momentIterationFunction and Algs. 1/2.
 *   - Time step: dt = CFL dx / a_max over all cells and nodes of the current
 *     ansatz (2D: CFL / (a_x/dx + a_y/dy)), last step clipped to t_end.
 *   - Rusanov speed per node pair: max(|v_n|+c) of the two node states.
 *   - 2D: unsplit five-point finite-volume update with normal fluxes.
 *   - IC cell average: midpoint (cell-centre) sampling.
 *   - Initial dual: projection of the entropy variables, then converged.
 *   - Multi-index order: total degree ascending, then first exponent
 *     descending (gives the prefix property used by per-cell degrees).
 *   - Steady residual (eq:residualSteady): Euclidean norm over all N*m
 *     moments, weighted by the cell volume.
 *   - Adaptivity (Sec. 5, Alg. ad-IPM): levels are total degrees; the
 *     indicator is taken on the first conserved variable of the ansatz
 *     u_s(lambda^T phi) at the cell's current level, right after its dual
 *     solve; one level per step; the printed thresholds are ordered
 *     delta_lo < delta_hi (lower below the smaller, raise above the larger);
 *     one quadrature rule serves every level (its nodes contain those of
 *     every coarser level trivially), so a neighbour's ansatz is read at
 *     the shared nodes whatever its level.
 *   - Refinement retardation (Alg. adosIPM): the printed cap takes the max of
 *     the determined level and the stage's level; the text calls the stage's
 *     level the maximal one, so the level is the min of the two.  The stage
 *     test follows the steady stop test of the same step; the steady stop
 *     applies only in the last stage.
 */
#include "ipm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Quadrature and basis (Sec. 2; eq:numberBasisFcts; App. A table A)   */
/* ------------------------------------------------------------------ */

int orc_num_basis(int p, int degree)
{
  /* N = binomial(M + p, p), eq:numberBasisFcts */
  long long r = 1;
  for (int k = 1; k <= p; ++k) r = r * (degree + k) / k;
  return (int)r;
}

/* Legendre P_n(x) and P_n'(x) by the three-term recurrence. */
static void legendre_and_derivative(int n, double x, double *pn, double *dpn)
{
  double p0 = 1.0, p1 = x;
  if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

static double legendre(int n, double x)
{
  double p0 = 1.0, p1 = x;
  if (n == 0) return 1.0;
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

/* n-point Gauss-Legendre rule on [-1,1], nodes ascending, weights sum 2:
   Newton's method on P_n from the Chebyshev-like guesses, then
   w = 2 / ((1 - x^2) P_n'(x)^2). */
int orc_gauss_legendre(int n, double *x, double *w)
{
  if (n < 1) return -1;
  for (int k = 0; k < n; ++k) {
    double z = cos(M_PI * (k + 0.75) / (n + 0.5));
    double pn, dpn;
    for (int it = 0; it < 100; ++it) {
      legendre_and_derivative(n, z, &pn, &dpn);
      double dz = pn / dpn;
      z -= dz;
      if (fabs(dz) <= 1e-16) break;
    }
    legendre_and_derivative(n, z, &pn, &dpn);
    x[n - 1 - k] = z;
    w[n - 1 - k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  return n;
}

/* Tensor rule for xi ~ U(-1,1)^p: node q = ((q_1 * n + q_2) * n + ...) with
   q_1 slowest; weight w_q f_Xi(xi_q) = prod w_{q_k} / 2 (Sec. 3.1, quadrature
   <h>_Q includes the density), so the weights sum to one. */
int orc_quadrature(int p, int qpd, double *nodes, double *w)
{
  double x[256], wx[256];
  if (p < 1 || qpd < 1 || qpd > 256) return -1;
  orc_gauss_legendre(qpd, x, wx);
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= qpd;
  for (int q = 0; q < Q; ++q) {
    int rem = q;
    double wt = 1.0;
    for (int k = p - 1; k >= 0; --k) {
      int ik = rem % qpd;
      rem /= qpd;
      nodes[q * p + k] = x[ik];
      wt *= 0.5 * wx[ik];
    }
    w[q] = wt;
  }
  return Q;
}

/* Clenshaw-Curtis: nodes cos(pi k/(n-1)) (ascending), weights as the
   integrals over [-1, 1] of the Lagrange polynomials of the nodes, each
   integrated by Gauss-Legendre (exact: degree n-1).  n = 1: midpoint.
   w = NULL: nodes only. */
int orc_clenshaw_curtis(int n, double *x, double *w)
{
  if (n < 1) return 0;
  if (n == 1) {
    x[0] = 0.0;
    if (w) w[0] = 2.0;
    return 1;
  }
  for (int k = 0; k < n; ++k) x[k] = -cos(M_PI * k / (n - 1));
  x[0] = -1.0;
  x[n - 1] = 1.0;
  if ((n - 1) % 2 == 0) x[(n - 1) / 2] = 0.0;
  if (!w) return n;
  double *gx = (double *)malloc(sizeof(double) * n), *gw = (double *)malloc(sizeof(double) * n);
  orc_gauss_legendre(n, gx, gw);
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int q = 0; q < n; ++q) {
      double l = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != k) l *= (gx[q] - x[j]) / (x[k] - x[j]);
      s += gw[q] * l;
    }
    w[k] = s;
  }
  free(gx);
  free(gw);
  return n;
}

/* one contribution to a sparse grid: fine-grid indices packed in a key */
typedef struct {
  long long key;
  double w;
} contrib_t;

static int cmp_contrib(const void *a, const void *b)
{
  long long ka = ((const contrib_t *)a)->key, kb = ((const contrib_t *)b)->key;
  return ka < kb ? -1 : ka > kb ? 1 : 0;
}

/* Smolyak sparse grid of level L from the nested Clenshaw-Curtis rules U_l
   with m(1) = 1, m(l) = 2^(l-1) + 1 points, as the sum over multi-levels
   l_1 + ... + l_p <= L + p of the tensor products of the difference rules
   D_l = U_l - U_(l-1) (U_0 = 0).  Every node lies on the finest grid
   (2^L + 1 points per dimension); contributions are merged on it.  If
   nodes is NULL only the node count is returned. */
static int cc_sparse(int p, int L, double *nodes, double *wts)
{
  int fine = (1 << L) + 1;
  double *xf = (double *)malloc(sizeof(double) * fine);
  orc_clenshaw_curtis(fine, xf, NULL);
  /* 1D difference rules on fine indices: dn[l], di[l][], dw[l][] */
  int Lmax = L + 1;
  int *dn = (int *)calloc(Lmax + 1, sizeof(int));
  int **di = (int **)calloc(Lmax + 1, sizeof(int *));
  double **dw = (double **)calloc(Lmax + 1, sizeof(double *));
  for (int l = 1; l <= Lmax; ++l) {
    di[l] = (int *)calloc(fine, sizeof(int));
    dw[l] = (double *)calloc(fine, sizeof(double));
    double *acc = (double *)calloc(fine, sizeof(double));
    char *used = (char *)calloc(fine, 1);
    for (int sgn = 0; sgn < 2; ++sgn) {
      int lev = l - sgn;
      if (lev < 1) continue;
      int m = lev == 1 ? 1 : (1 << (lev - 1)) + 1;
      double *x = (double *)malloc(sizeof(double) * m), *w = (double *)calloc(m, sizeof(double));
      orc_clenshaw_curtis(m, x, nodes ? w : NULL);  /* counting needs no weights */
      for (int k = 0; k < m; ++k) {
        int g = m == 1 ? (fine - 1) / 2 : k * ((fine - 1) / (m - 1));
        acc[g] += (sgn ? -1.0 : 1.0) * 0.5 * w[k];
        used[g] = 1;
      }
      free(x);
      free(w);
    }
    for (int g = 0; g < fine; ++g)
      if (used[g]) {
        di[l][dn[l]] = g;
        dw[l][dn[l]] = acc[g];
        dn[l]++;
      }
    free(acc);
    free(used);
  }
  size_t cap = 1024, cnt = 0;
  contrib_t *c = (contrib_t *)malloc(sizeof(contrib_t) * cap);
  int lv[3] = {1, 1, 1};
  for (;;) {
    int s = 0;
    for (int d = 0; d < p; ++d) s += lv[d];
    if (s <= L + p) {
      int ix[3] = {0, 0, 0};
      for (;;) {
        long long key = 0;
        double w = 1.0;
        for (int d = 0; d < p; ++d) {
          key = key * fine + di[lv[d]][ix[d]];
          w *= dw[lv[d]][ix[d]];
        }
        if (cnt == cap) {
          cap *= 2;
          c = (contrib_t *)realloc(c, sizeof(contrib_t) * cap);
        }
        c[cnt].key = key;
        c[cnt].w = w;
        cnt++;
        int d = p - 1;
        while (d >= 0 && ++ix[d] == dn[lv[d]]) ix[d--] = 0;
        if (d < 0) break;
      }
    }
    int d = p - 1;
    while (d >= 0 && ++lv[d] > Lmax) lv[d--] = 1;
    if (d < 0) break;
  }
  qsort(c, cnt, sizeof(contrib_t), cmp_contrib);
  int Q = 0;
  for (size_t i = 0; i < cnt;) {
    size_t j = i;
    double w = 0.0;
    while (j < cnt && c[j].key == c[i].key) w += c[j++].w;
    if (nodes) {
      long long r = c[i].key;
      for (int d = p - 1; d >= 0; --d) {
        nodes[(size_t)Q * p + d] = xf[r % fine];
        r /= fine;
      }
      wts[Q] = w;
    }
    Q++;
    i = j;
  }
  free(c);
  for (int l = 1; l <= Lmax; ++l) {
    free(di[l]);
    free(dw[l]);
  }
  free(dn);
  free(di);
  free(dw);
  free(xf);
  return Q;
}

int orc_quadrature_size(int rule, int p, int param)
{
  if (p < 1 || p > 3) return 0;
  if (rule == ORC_QUAD_CC_SPARSE) return param >= 0 ? cc_sparse(p, param, NULL, NULL) : 0;
  if (param < 1) return 0;
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= param;
  return Q;
}

int orc_quadrature_rule(int rule, int p, int param, double *nodes, double *w)
{
  if (rule == ORC_QUAD_GL) return orc_quadrature(p, param, nodes, w);
  if (rule == ORC_QUAD_CC_SPARSE) return cc_sparse(p, param, nodes, w);
  /* tensor Clenshaw-Curtis, first coordinate slowest, weights / 2 per dim */
  double *x = (double *)malloc(sizeof(double) * param), *w1 = (double *)malloc(sizeof(double) * param);
  orc_clenshaw_curtis(param, x, w1);
  int Q = orc_quadrature_size(rule, p, param);
  for (int q = 0; q < Q; ++q) {
    int r = q;
    w[q] = 1.0;
    for (int k = p - 1; k >= 0; --k) {
      int d = r % param;
      r /= param;
      nodes[(size_t)q * p + k] = x[d];
      w[q] *= 0.5 * w1[d];
    }
  }
  free(x);
  free(w1);
  return Q;
}

static void gen_indices(int p, int left, int pos, int *cur, int *out, int *cnt)
{
  if (pos == p - 1) {
    cur[pos] = left;
    for (int k = 0; k < p; ++k) out[(*cnt) * p + k] = cur[k];
    ++*cnt;
    return;
  }
  for (int e = left; e >= 0; --e) {
    cur[pos] = e;
    gen_indices(p, left - e, pos + 1, cur, out, cnt);
  }
}

/* Multi-indices with |i| <= M (Sec. 2), graded: total degree ascending,
   first exponent descending within a degree. */
int orc_multi_indices(int p, int degree, int *idx)
{
  int cur[16], cnt = 0;
  if (p < 1 || p > 16) return -1;
  for (int d = 0; d <= degree; ++d) gen_indices(p, d, 0, cur, idx, &cnt);
  return cnt;
}

/* Phi[q][i] = phi_i(xi_q), phi_i = prod_k sqrt(2 i_k + 1) P_{i_k}(xi_k):
   orthonormal under the uniform density (Sec. 2, gPC basis). */
void orc_basis_eval(int p, int degree, int Q, const double *nodes, double *Phi)
{
  int N = orc_num_basis(p, degree);
  int *idx = (int *)malloc(sizeof(int) * N * p);
  orc_multi_indices(p, degree, idx);
  for (int q = 0; q < Q; ++q)
    for (int i = 0; i < N; ++i) {
      double v = 1.0;
      for (int k = 0; k < p; ++k) {
        int e = idx[i * p + k];
        v *= sqrt(2.0 * e + 1.0) * legendre(e, nodes[q * p + k]);
      }
      Phi[q * N + i] = v;
    }
  free(idx);
}

/* eq:errorIndicator: the truncations u_l are evaluated at the nodes and the
   averages are quadrature sums, exactly as the definition reads. */
void orc_indicator(int p, int L, int qpd, const double *u_nodes, double *S)
{
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= qpd;
  double *nodes = (double *)malloc(sizeof(double) * Q * p);
  double *w = (double *)malloc(sizeof(double) * Q);
  orc_quadrature(p, qpd, nodes, w);
  int N = orc_num_basis(p, L);
  double *Phi = (double *)malloc(sizeof(double) * Q * N);
  double *uh = (double *)malloc(sizeof(double) * N);
  double *prev = (double *)malloc(sizeof(double) * Q);
  double *cur = (double *)malloc(sizeof(double) * Q);
  orc_basis_eval(p, L, Q, nodes, Phi);
  for (int i = 0; i < N; ++i) {
    double a = 0.0;
    for (int q = 0; q < Q; ++q) a += w[q] * u_nodes[q] * Phi[q * N + i];
    uh[i] = a;
  }
  for (int q = 0; q < Q; ++q) prev[q] = uh[0] * Phi[q * N];  /* u_0 */
  for (int l = 1; l <= L; ++l) {
    int Nl = orc_num_basis(p, l);
    double num = 0.0, den = 0.0;
    for (int q = 0; q < Q; ++q) {
      double v = 0.0;
      for (int i = 0; i < Nl; ++i) v += uh[i] * Phi[q * N + i];
      cur[q] = v;
      num += w[q] * (v - prev[q]) * (v - prev[q]);
      den += w[q] * v * v;
    }
    S[l - 1] = num / den;
    for (int q = 0; q < Q; ++q) prev[q] = cur[q];
  }
  free(nodes);
  free(w);
  free(Phi);
  free(uh);
  free(prev);
  free(cur);
}

void orc_select_degrees(int p, int L, int qpd, int m, int cells, const double *ic_nodal,
                        double delta_hi, signed char *out)
{
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= qpd;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < cells; ++c) {
    double u[1024], S[16];
    double *uu = Q <= (int)(sizeof(u) / sizeof(u[0])) ? u : (double *)malloc(sizeof(double) * Q);
    for (int q = 0; q < Q; ++q) uu[q] = ic_nodal[((size_t)c * Q + q) * m];
    orc_indicator(p, L, qpd, uu, S);
    int lev = 1;
    for (int l = 2; l <= L; ++l)
      if (S[l - 1] > delta_hi) lev = l;
    out[c] = (signed char)lev;
    if (uu != u) free(uu);
  }
}

/* ------------------------------------------------------------------ */
/* Closures u_s = (grad s)^-1, its Jacobian, s_* (Sec. 2 eq:ansatz,     */
/* Sec. 3.1; App. B for Euler)                                          */
/* ------------------------------------------------------------------ */

/* Returns 1 if Lam lies in the closure's domain. J is the full m x m
   Jacobian of u_s, sstar the Legendre dual s_*(Lam). */
int orc_closure(int entropy, int m, double gamma, double um, double up,
                const double *Lam, double *u, double *J, double *sstar)
{
  if (entropy == ORC_ENT_QUADRATIC) {
    /* s(u) = |u|^2/2: u_s = Lam, grad u_s = I, s_* = |Lam|^2/2 */
    double s = 0.0;
    for (int a = 0; a < m; ++a) {
      u[a] = Lam[a];
      s += 0.5 * Lam[a] * Lam[a];
      for (int b = 0; b < m; ++b) J[a * m + b] = (a == b) ? 1.0 : 0.0;
    }
    *sstar = s;
    /* gas dynamics: a stochastic-Galerkin state with a non-positive density
       or pressure at a node has no physical flux (the failure of SG noted in
       Sec. 7); it is reported as inadmissible */
    if (m >= 3) {
      double mm = 0.0;
      for (int k = 1; k < m - 1; ++k) mm += u[k] * u[k];
      if (!(u[0] > 0.0)) return 0;
      if (!((gamma - 1.0) * (u[m - 1] - 0.5 * mm / u[0]) > 0.0)) return 0;
    }
    return 1;
  }
  if (entropy == ORC_ENT_LOG_BARRIER) {
    /* s(u) = (u-u-)ln(u-u-) + (u+-u)ln(u+-u): s'(u) = ln((u-u-)/(u+-u)),
       u_s = u- + D sigma(Lam), u_s' = D sigma (1-sigma),
       s_*(Lam) = u- Lam + D softplus(Lam) - D ln D,  D = u+ - u-. */
    double D = up - um, L = Lam[0], sig, oms;
    if (L >= 0.0) {
      double e = exp(-L);
      sig = 1.0 / (1.0 + e);
      oms = e / (1.0 + e);
    } else {
      double e = exp(L);
      sig = e / (1.0 + e);
      oms = 1.0 / (1.0 + e);
    }
    u[0] = um + D * sig;
    J[0] = D * sig * oms;
    double softplus = (L > 0.0 ? L : 0.0) + log1p(exp(-fabs(L)));
    *sstar = um * L + D * softplus - D * log(D);
    return 1;
  }
  /* Euler entropy s = -rho ln(rho^-gamma (E - |m|^2/(2 rho))), App. B.
     With beta = -Lam_E > 0, v = Lam_m / beta, e = 1/beta:
       ln rho = (ln beta - |Lam_m|^2/(2 beta) + gamma - Lam_rho) / (1 - gamma),
       m = rho v, E = rho (|v|^2/2 + e),
     Jacobian = rho/(gamma-1) w w^T + rho e (sum_k a_k a_k^T + e eE eE^T),
       w = (1, v, h), h = E/rho, a_k = (0, unit_k, v_k), eE = (0,..,0,1),
     and s_* = (gamma - 1) rho. */
  {
    int d = m - 2;
    double beta = -Lam[m - 1];
    if (!(beta > 0.0)) return 0;
    double v[2] = {0.0, 0.0}, vv = 0.0, lm2 = 0.0;
    for (int k = 0; k < d; ++k) {
      v[k] = Lam[1 + k] / beta;
      vv += v[k] * v[k];
      lm2 += Lam[1 + k] * Lam[1 + k];
    }
    double lnrho = (log(beta) - lm2 / (2.0 * beta) + gamma - Lam[0]) / (1.0 - gamma);
    double rho = exp(lnrho);
    double e = 1.0 / beta;
    double h = 0.5 * vv + e;
    u[0] = rho;
    for (int k = 0; k < d; ++k) u[1 + k] = rho * v[k];
    u[m - 1] = rho * h;
    double wv[ORC_MAXM];
    wv[0] = 1.0;
    for (int k = 0; k < d; ++k) wv[1 + k] = v[k];
    wv[m - 1] = h;
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) J[a * m + b] = rho / (gamma - 1.0) * wv[a] * wv[b];
    for (int k = 0; k < d; ++k) {
      double ak[ORC_MAXM] = {0.0, 0.0, 0.0, 0.0};
      ak[1 + k] = 1.0;
      ak[m - 1] = v[k];
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) J[a * m + b] += rho * e * ak[a] * ak[b];
    }
    J[(m - 1) * m + (m - 1)] += rho * e * e;
    *sstar = (gamma - 1.0) * rho;
    return isfinite(rho) ? 1 : 0;
  }
}

/* grad_u s(u) (entropy variables), used for the initial dual state. */
int orc_entropy_grad(int entropy, int m, double gamma, double um, double up,
                     const double *u, double *Lam)
{
  if (entropy == ORC_ENT_QUADRATIC) {
    for (int a = 0; a < m; ++a) Lam[a] = u[a];
    return 1;
  }
  if (entropy == ORC_ENT_LOG_BARRIER) {
    if (!(u[0] > um && u[0] < up)) return 0;
    Lam[0] = log((u[0] - um) / (up - u[0]));
    return 1;
  }
  {
    /* App. B, with the E-derivative read as -rho/eps:
       ds/drho = -ln(rho^-gamma eps) - |m|^2/(2 rho eps) + gamma,
       ds/dm   = m / eps,   ds/dE = -rho / eps,   eps = E - |m|^2/(2 rho) */
    int d = m - 2;
    double rho = u[0], mm = 0.0;
    for (int k = 0; k < d; ++k) mm += u[1 + k] * u[1 + k];
    double eps = u[m - 1] - mm / (2.0 * rho);
    if (!(rho > 0.0 && eps > 0.0)) return 0;
    Lam[0] = -log(pow(rho, -gamma) * eps) - mm / (2.0 * rho * eps) + gamma;
    for (int k = 0; k < d; ++k) Lam[1 + k] = u[1 + k] / eps;
    Lam[m - 1] = -rho / eps;
    return 1;
  }
}

double orc_entropy(int entropy, int m, double gamma, double um, double up, const double *u)
{
  if (entropy == ORC_ENT_QUADRATIC) {
    double s = 0.0;
    for (int a = 0; a < m; ++a) s += 0.5 * u[a] * u[a];
    return s;
  }
  if (entropy == ORC_ENT_LOG_BARRIER)
    return (u[0] - um) * log(u[0] - um) + (up - u[0]) * log(up - u[0]);
  {
    int d = m - 2;
    double rho = u[0], mm = 0.0;
    for (int k = 0; k < d; ++k) mm += u[1 + k] * u[1 + k];
    double eps = u[m - 1] - mm / (2.0 * rho);
    return -rho * log(pow(rho, -gamma) * eps);
  }
}

/* ------------------------------------------------------------------ */
/* Physical flux, wave speed, numerical fluxes                          */
/* ------------------------------------------------------------------ */

/* physical flux f(u) in direction dir (0 = x, 1 = y) and the spectral
   radius of its Jacobian (|u| for Burgers; |v_n| + c for Euler) */
static void phys_flux(int equation, int m, double gamma, int dir, const double *u,
                      double *f, double *speed)
{
  if (equation == ORC_BURGERS_1D) {
    f[0] = 0.5 * u[0] * u[0];
    *speed = fabs(u[0]);
    return;
  }
  int d = m - 2;
  double rho = u[0], vv = 0.0, v[2] = {0.0, 0.0};
  for (int k = 0; k < d; ++k) {
    v[k] = u[1 + k] / rho;
    vv += v[k] * v[k];
  }
  double E = u[m - 1];
  double p = (gamma - 1.0) * (E - 0.5 * rho * vv);
  double vn = v[dir];
  f[0] = rho * vn;
  for (int k = 0; k < d; ++k) f[1 + k] = u[1 + k] * vn + (k == dir ? p : 0.0);
  f[m - 1] = (E + p) * vn;
  *speed = fabs(vn) + sqrt(gamma * p / rho);
}

/* deterministic numerical flux g(u_l, u_r) (Sec. 3.1, kinetic flux input):
   Lax-Friedrichs  g = (f_l + f_r)/2 - dx/(2 dt) (u_r - u_l)  (App. A),
   Rusanov         g = (f_l + f_r)/2 - max(a_l, a_r)/2 (u_r - u_l). */
static void num_flux(const orc_state *S, int dir, const double *ul, const double *ur,
                     double dt, double *g);

/* ------------------------------------------------------------------ */
/* State                                                                */
/* ------------------------------------------------------------------ */

struct orc_state {
  orc_problem pb;
  int m, N, Q, cells, n, dim;
  double dx, dy, vol;
  double *nodes, *w, *Phi;
  int *Nc;                 /* modes per cell (prefix of the graded basis) */
  int *deg, *deg_next;     /* total degree per cell: this step, next step */
  double *uhat, *lam, *unew, *nodal; /* [cells][m][N] x3, [cells][Q][m] */
  double *ghost[4];        /* Dirichlet ghost nodal states [Q][m] */
  double *Ctp;             /* [N][N][N] <phi_i phi_n phi_k> (analytic SG flux) */
  int *iters;
  orc_info info;
};

static void num_flux(const orc_state *S, int dir, const double *ul, const double *ur,
                     double dt, double *g)
{
  int m = S->m;
  double fl[ORC_MAXM], fr[ORC_MAXM], al, ar;
  phys_flux(S->pb.equation, m, S->pb.gamma, dir, ul, fl, &al);
  phys_flux(S->pb.equation, m, S->pb.gamma, dir, ur, fr, &ar);
  double h = dir == 0 ? S->dx : S->dy;
  double visc = S->pb.flux == ORC_FLUX_LF ? h / (2.0 * dt) : 0.5 * (al > ar ? al : ar);
  for (int a = 0; a < m; ++a) g[a] = 0.5 * (fl[a] + fr[a]) - visc * (ur[a] - ul[a]);
}

/* ------------------------------------------------------------------ */
/* Dual problem of one cell (eq:L, eq:dualIterationFunction, eq:tauCrit) */
/* ------------------------------------------------------------------ */

/* Ansatz at every node for lam (layout [m][N], first Nl modes used):
   u[q][a], J[q][a][b], sstar[q].  Returns 0 if some node is inadmissible. */
static int eval_nodes(const orc_state *S, int Nl, const double *lam, double *u, double *J,
                      double *ss)
{
  int m = S->m, N = S->N;
  for (int q = 0; q < S->Q; ++q) {
    double Lam[ORC_MAXM];
    for (int a = 0; a < m; ++a) {
      double s = 0.0;
      for (int i = 0; i < Nl; ++i) s += lam[a * N + i] * S->Phi[q * N + i];
      Lam[a] = s;
    }
    if (!orc_closure(S->pb.entropy, m, S->pb.gamma, S->pb.u_minus, S->pb.u_plus, Lam,
                     u + q * m, J + q * m * m, ss + q))
      return 0;
  }
  return 1;
}

/* L(lam; uhat) = <s_*(lam^T phi)>_Q - sum_i lam_i^T uhat_i   (eq:L) */
static double dual_cost_from_nodes(const orc_state *S, int Nl, const double *lam,
                                   const double *uhat, const double *ss)
{
  double L = 0.0;
  for (int q = 0; q < S->Q; ++q) L += S->w[q] * ss[q];
  for (int a = 0; a < S->m; ++a)
    for (int i = 0; i < Nl; ++i) L -= lam[a * S->N + i] * uhat[a * S->N + i];
  return L;
}

/* grad L = <u_s(lam^T phi) phi^T>_Q^T - uhat, stored compactly [m][Nl] */
static void dual_gradient(const orc_state *S, int Nl, const double *u, const double *uhat,
                          double *g)
{
  int m = S->m, N = S->N;
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < Nl; ++i) {
      double s = 0.0;
      for (int q = 0; q < S->Q; ++q) s += S->w[q] * u[q * m + a] * S->Phi[q * N + i];
      g[a * Nl + i] = s - uhat[a * N + i];
    }
}

/* H = <grad u_s(lam^T phi) (x) phi phi^T>_Q, compact [(a,i)][(b,k)] */
static void dual_hessian(const orc_state *S, int Nl, const double *J, double *H)
{
  int m = S->m, N = S->N, n = m * Nl;
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < Nl; ++i)
      for (int b = 0; b < m; ++b)
        for (int k = 0; k < Nl; ++k) {
          double s = 0.0;
          for (int q = 0; q < S->Q; ++q)
            s += S->w[q] * J[(q * m + a) * m + b] * S->Phi[q * N + i] * S->Phi[q * N + k];
          H[(a * Nl + i) * n + (b * Nl + k)] = s;
        }
}

/* Cholesky H = L L^T in place (lower), then solve H d = g. 0 on failure. */
static int cholesky_solve(int n, double *H, const double *g, double *d)
{
  for (int j = 0; j < n; ++j) {
    double s = H[j * n + j];
    for (int k = 0; k < j; ++k) s -= H[j * n + k] * H[j * n + k];
    if (!(s > 0.0)) return 0;
    double ljj = sqrt(s);
    H[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = H[i * n + j];
      for (int k = 0; k < j; ++k) t -= H[i * n + k] * H[j * n + k];
      H[i * n + j] = t / ljj;
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = g[i];
    for (int k = 0; k < i; ++k) s -= H[i * n + k] * d[k];
    d[i] = s / H[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = d[i];
    for (int k = i + 1; k < n; ++k) s -= H[k * n + i] * d[k];
    d[i] = s / H[i * n + i];
  }
  return 1;
}

typedef struct {
  double *u, *J, *ss, *g, *H, *d, *trial;
} scratch_t;

static scratch_t scratch_alloc(const orc_state *S)
{
  scratch_t w;
  int Q = S->Q, m = S->m, n = S->n;
  w.u = (double *)malloc(sizeof(double) * Q * m);
  w.J = (double *)malloc(sizeof(double) * Q * m * m);
  w.ss = (double *)malloc(sizeof(double) * Q);
  w.g = (double *)malloc(sizeof(double) * n);
  w.H = (double *)malloc(sizeof(double) * n * n);
  w.d = (double *)malloc(sizeof(double) * n);
  w.trial = (double *)malloc(sizeof(double) * m * S->N);
  return w;
}

static void scratch_free(scratch_t *w)
{
  free(w->u); free(w->J); free(w->ss); free(w->g); free(w->H); free(w->d); free(w->trial);
}

/* Newton iteration lambda <- d(lambda, uhat) (eq:dualIterationFunction).
   one_shot = 0: iterate until eq:tauCrit holds (Alg. 1), with the
   backtracking rule described at the top of this file.
   one_shot = 1: exactly one full step (eq:oneshotIPMdual, Alg. 2).
   Returns status bits; *iters = number of Newton updates taken. */
static int dual_newton(const orc_state *S, int Nl, const double *uhat, double *lam,
                       int one_shot, int *iters, scratch_t *w)
{
  int m = S->m, N = S->N, n = m * Nl, st = 0;
  for (int it = 0;; ++it) {
    *iters = it;
    if (!eval_nodes(S, Nl, lam, w->u, w->J, w->ss)) return st | ORC_ST_REALIZABILITY;
    dual_gradient(S, Nl, w->u, uhat, w->g);
    double r = 0.0;
    for (int a = 0; a < m; ++a) {
      double s2 = 0.0;
      for (int i = 0; i < Nl; ++i) s2 += w->g[a * Nl + i] * w->g[a * Nl + i];
      r += sqrt(s2);
    }
    if (!isfinite(r)) return st | ORC_ST_NONFINITE;
    if (!one_shot) {
      if (r < S->pb.tau) return st;
      if (it >= S->pb.max_newton) return st | ORC_ST_NEWTON;
    }
    dual_hessian(S, Nl, w->J, w->H);
    if (!cholesky_solve(n, w->H, w->g, w->d)) return st | ORC_ST_CHOLESKY;
    double t = 1.0;
    if (!one_shot && r > 1e-6) {
      double L0 = dual_cost_from_nodes(S, Nl, lam, uhat, w->ss);
      double slope = 0.0;
      for (int k = 0; k < n; ++k) slope += w->g[k] * w->d[k];
      for (int h = 0;; ++h) {
        memcpy(w->trial, lam, sizeof(double) * m * N);
        for (int a = 0; a < m; ++a)
          for (int i = 0; i < Nl; ++i) w->trial[a * N + i] -= t * w->d[a * Nl + i];
        int ok = eval_nodes(S, Nl, w->trial, w->u, w->J, w->ss);
        if (ok) {
          double Lt = dual_cost_from_nodes(S, Nl, w->trial, uhat, w->ss);
          if (Lt <= L0 - 1e-4 * t * slope) break;
        }
        if (h == 60) return st | ORC_ST_LINESEARCH;
        t *= 0.5;
      }
    }
    for (int a = 0; a < m; ++a)
      for (int i = 0; i < Nl; ++i) lam[a * N + i] -= t * w->d[a * Nl + i];
    if (one_shot) {
      *iters = 1;
      return st;
    }
  }
}

/* nodal values u_s(lam^T phi_q) of one cell, [Q][m] */
static int cell_nodal(const orc_state *S, int Nl, const double *lam, double *out)
{
  int m = S->m;
  for (int q = 0; q < S->Q; ++q) {
    double Lam[ORC_MAXM], J[ORC_MAXM * ORC_MAXM], ss;
    for (int a = 0; a < m; ++a) {
      double s = 0.0;
      for (int i = 0; i < Nl; ++i) s += lam[a * S->N + i] * S->Phi[q * S->N + i];
      Lam[a] = s;
    }
    if (!orc_closure(S->pb.entropy, m, S->pb.gamma, S->pb.u_minus, S->pb.u_plus, Lam,
                     out + q * m, J, &ss))
      return 0;
  }
  return 1;
}

/* projection <v phi_i>_Q of nodal values [Q][m] onto the first Nl modes */
static void project(const orc_state *S, int Nl, const double *nodal, double *mom)
{
  int m = S->m, N = S->N;
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      if (i < Nl)
        for (int q = 0; q < S->Q; ++q) s += S->w[q] * nodal[q * m + a] * S->Phi[q * N + i];
      mom[a * N + i] = s;
    }
}

/* initial dual: projection of the entropy variables grad s(u_IC) (then the
   caller converges it) */
static int initial_dual(const orc_state *S, int Nl, const double *nodal, double *lam)
{
  int m = S->m, N = S->N, Q = S->Q;
  double *ev = (double *)malloc(sizeof(double) * Q * m);
  int ok = 1;
  for (int q = 0; q < Q; ++q)
    ok &= orc_entropy_grad(S->pb.entropy, m, S->pb.gamma, S->pb.u_minus, S->pb.u_plus,
                           nodal + q * m, ev + q * m);
  project(S, Nl, ev, lam);
  (void)N;
  free(ev);
  return ok;
}

/* ------------------------------------------------------------------ */
/* Problem setup                                                        */
/* ------------------------------------------------------------------ */

int orc_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

orc_state *orc_create(const orc_problem *pb, const signed char *cell_degree,
                      const double *ic_nodal, const double *dirichlet_nodal)
{
  orc_state *S = (orc_state *)calloc(1, sizeof(orc_state));
  S->pb = *pb;
  S->dim = pb->equation == ORC_EULER_2D ? 2 : 1;
  S->m = pb->equation == ORC_BURGERS_1D ? 1 : (pb->equation == ORC_EULER_1D ? 3 : 4);
  if (S->dim == 1) S->pb.ny = 1;
  S->N = orc_num_basis(pb->p, pb->degree);
  S->n = S->m * S->N;
  int Q = orc_quadrature_size(pb->quad_rule, pb->p, pb->quad_per_dim);
  S->Q = Q;
  S->cells = S->pb.nx * S->pb.ny;
  S->dx = (pb->x1 - pb->x0) / pb->nx;
  S->dy = S->dim == 2 ? (pb->y1 - pb->y0) / pb->ny : 1.0;
  S->vol = S->dim == 2 ? S->dx * S->dy : S->dx;
  S->nodes = (double *)malloc(sizeof(double) * Q * pb->p);
  S->w = (double *)malloc(sizeof(double) * Q);
  S->Phi = (double *)malloc(sizeof(double) * Q * S->N);
  orc_quadrature_rule(pb->quad_rule, pb->p, pb->quad_per_dim, S->nodes, S->w);
  orc_basis_eval(pb->p, pb->degree, Q, S->nodes, S->Phi);
  if (pb->flux == ORC_FLUX_SG_ANALYTIC) {
    /* App. A: C_i = <phi phi^T phi_i>, integrands of degree <= 3M, by a
       tensor Gauss-Legendre rule exact to that degree */
    int qc = (3 * pb->degree) / 2 + 1, Qc = 1;
    for (int k = 0; k < pb->p; ++k) Qc *= qc;
    double *nc = (double *)malloc(sizeof(double) * Qc * pb->p);
    double *wc = (double *)malloc(sizeof(double) * Qc);
    double *Pc = (double *)malloc(sizeof(double) * Qc * S->N);
    orc_quadrature(pb->p, qc, nc, wc);
    orc_basis_eval(pb->p, pb->degree, Qc, nc, Pc);
    int N = S->N;
    S->Ctp = (double *)calloc((size_t)N * N * N, sizeof(double));
    for (int i = 0; i < N; ++i)
      for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
          double t = 0.0;
          for (int q = 0; q < Qc; ++q) t += wc[q] * Pc[q * N + i] * Pc[q * N + a] * Pc[q * N + b];
          S->Ctp[((size_t)i * N + a) * N + b] = t;
        }
    free(nc);
    free(wc);
    free(Pc);
  }
  size_t cn = (size_t)S->cells * S->n;
  S->uhat = (double *)calloc(cn, sizeof(double));
  S->lam = (double *)calloc(cn, sizeof(double));
  S->unew = (double *)calloc(cn, sizeof(double));
  S->nodal = (double *)calloc((size_t)S->cells * Q * S->m, sizeof(double));
  S->iters = (int *)calloc(S->cells, sizeof(int));
  S->Nc = (int *)malloc(sizeof(int) * S->cells);
  S->deg = (int *)malloc(sizeof(int) * S->cells);
  S->deg_next = (int *)malloc(sizeof(int) * S->cells);
  for (int c = 0; c < S->cells; ++c) {
    S->deg[c] = cell_degree ? cell_degree[c] : pb->degree;
    S->Nc[c] = orc_num_basis(pb->p, S->deg[c]);
  }

  int st = 0;
  /* IC (Alg. 1, first loop): uhat_j^0 = <u_IC(x_j, .) phi>_Q at cell centres,
     then the dual of the IC moments, converged */
#pragma omp parallel reduction(| : st)
  {
    scratch_t w = scratch_alloc(S);
#pragma omp for schedule(static)
    for (int c = 0; c < S->cells; ++c) {
      const double *nod = ic_nodal + (size_t)c * Q * S->m;
      project(S, S->Nc[c], nod, S->uhat + (size_t)c * S->n);
      if (!initial_dual(S, S->Nc[c], nod, S->lam + (size_t)c * S->n)) st |= ORC_ST_REALIZABILITY;
      int k;
      st |= dual_newton(S, S->Nc[c], S->uhat + (size_t)c * S->n, S->lam + (size_t)c * S->n, 0,
                        &k, &w);
    }
    scratch_free(&w);
  }
  /* Dirichlet ghosts: fixed moments, converged dual, their nodal ansatz */
  for (int side = 0; side < 4; ++side) {
    S->ghost[side] = NULL;
    if (pb->bc[side] != ORC_BC_DIRICHLET || !dirichlet_nodal) continue;
    if (S->dim == 1 && side >= 2) continue;
    const double *nod = dirichlet_nodal + (size_t)side * Q * S->m;
    double *gm = (double *)malloc(sizeof(double) * S->n);
    double *gl = (double *)malloc(sizeof(double) * S->n);
    scratch_t w = scratch_alloc(S);
    project(S, S->N, nod, gm);
    if (!initial_dual(S, S->N, nod, gl)) st |= ORC_ST_REALIZABILITY;
    int k;
    st |= dual_newton(S, S->N, gm, gl, 0, &k, &w);
    S->ghost[side] = (double *)malloc(sizeof(double) * Q * S->m);
    if (!cell_nodal(S, S->N, gl, S->ghost[side])) st |= ORC_ST_REALIZABILITY;
    scratch_free(&w);
    free(gm);
    free(gl);
  }
  S->info.status = st;
  return S;
}

void orc_destroy(orc_state *S)
{
  if (!S) return;
  free(S->nodes); free(S->w); free(S->Phi); free(S->uhat); free(S->lam); free(S->unew);
  free(S->nodal); free(S->iters); free(S->Nc); free(S->deg); free(S->deg_next); free(S->Ctp);
  for (int k = 0; k < 4; ++k) free(S->ghost[k]);
  free(S);
}

void orc_sizes(const orc_state *S, int *m, int *N, int *Q, int *cells)
{
  *m = S->m; *N = S->N; *Q = S->Q; *cells = S->cells;
}

/* neighbour's nodal values across side (0 x-, 1 x+, 2 y-, 3 y+) */
static const double *neighbour(const orc_state *S, int ix, int iy, int side)
{
  int nx = S->pb.nx, ny = S->pb.ny, jx = ix, jy = iy;
  if (side == 0) --jx;
  if (side == 1) ++jx;
  if (side == 2) --jy;
  if (side == 3) ++jy;
  int out = jx < 0 || jx >= nx || jy < 0 || jy >= ny;
  if (out) {
    int bc = S->pb.bc[side];
    if (bc == ORC_BC_PERIODIC) {
      jx = (jx + nx) % nx;
      jy = (jy + ny) % ny;
    } else if (bc == ORC_BC_DIRICHLET && S->ghost[side]) {
      return S->ghost[side];
    } else {
      jx = ix;
      jy = iy;
    }
  }
  return S->nodal + ((size_t)jy * nx + jx) * S->Q * S->m;
}

/* DetermineRefinementLevel of Alg. ad-IPM for cell c after its dual solve:
   the indicator eq:errorIndicator of the first conserved variable of the
   ansatz u_s(lam^T phi) at the cell's current level d (moments up to degree
   d and the averages by quadrature, orc_indicator); below delta_lo the cell
   goes one level down, above delta_hi one level up, kept within
   [min_degree, degree].  The thresholds are ordered delta_lo < delta_hi
   (the experiments of Sec. 7 print them the other way round). */
static int next_level(const orc_state *S, int c)
{
  int d = S->deg[c], Q = S->Q, m = S->m;
  double *u = (double *)malloc(sizeof(double) * Q);
  double *Sv = (double *)malloc(sizeof(double) * (d > 0 ? d : 1));
  for (int q = 0; q < Q; ++q) u[q] = S->nodal[((size_t)c * Q + q) * m];
  int dn = d;
  if (d >= 1) {
    orc_indicator(S->pb.p, d, S->pb.quad_per_dim, u, Sv);
    double ind = Sv[d - 1];
    if (ind < S->pb.delta_lo && d > S->pb.min_degree) dn = d - 1;
    else if (ind > S->pb.delta_hi && d < S->pb.degree) dn = d + 1;
  }
  free(u);
  free(Sv);
  return dn;
}

/* ------------------------------------------------------------------ */
/* Time stepping: Alg. 1 (IPM) and Alg. 2 (one-shot IPM)                */
/* ------------------------------------------------------------------ */

int orc_step(orc_state *S, int max_steps, orc_info *info)
{
  int m = S->m, Q = S->Q, n = S->n;
  for (int s = 0; s < max_steps && !S->info.done; ++s) {
    int st = 0, maxit = 0;
    long long its = 0;
    /* dual step for every cell: converged (Alg. 1) or one Newton step
       (Alg. 2); then the ansatz at the nodes */
#pragma omp parallel reduction(| : st) reduction(+ : its) reduction(max : maxit)
    {
      scratch_t w = scratch_alloc(S);
#pragma omp for schedule(dynamic, 16)
      for (int c = 0; c < S->cells; ++c) {
        int k = 0;
        st |= dual_newton(S, S->Nc[c], S->uhat + (size_t)c * n, S->lam + (size_t)c * n,
                          S->pb.one_shot, &k, &w);
        S->iters[c] = k;
        its += k;
        if (k > maxit) maxit = k;
        if (!cell_nodal(S, S->Nc[c], S->lam + (size_t)c * n, S->nodal + (size_t)c * Q * m))
          st |= ORC_ST_REALIZABILITY;
      }
      scratch_free(&w);
    }
    /* Alg. ad-IPM: the level of the next step from the new dual state;
       Alg. adosIPM: capped by the maximal level of the retardation stage */
    if (S->pb.adapt) {
      int cap = S->pb.n_retard > 0 ? S->pb.retard_degree[S->info.retard_stage] : S->pb.degree;
#pragma omp parallel for schedule(static)
      for (int c = 0; c < S->cells; ++c) {
        int dn = next_level(S, c);
        S->deg_next[c] = dn < cap ? dn : cap;
      }
    }
    /* time step from the largest wave speed over all cells and nodes */
    double ax = 0.0, ay = 0.0;
    for (int c = 0; c < S->cells + 4; ++c) {
      const double *nod;
      if (c < S->cells) nod = S->nodal + (size_t)c * Q * m;
      else if (S->ghost[c - S->cells]) nod = S->ghost[c - S->cells];
      else continue;
      for (int q = 0; q < Q; ++q) {
        double f[ORC_MAXM], a;
        phys_flux(S->pb.equation, m, S->pb.gamma, 0, nod + q * m, f, &a);
        if (!(a >= 0.0)) st |= ORC_ST_NONFINITE;
        if (a > ax) ax = a;
        if (S->dim == 2) {
          phys_flux(S->pb.equation, m, S->pb.gamma, 1, nod + q * m, f, &a);
          if (!(a >= 0.0)) st |= ORC_ST_NONFINITE;
          if (a > ay) ay = a;
        }
      }
    }
    double dt = S->dim == 2 ? S->pb.cfl / (ax / S->dx + ay / S->dy) : S->pb.cfl * S->dx / ax;
    int last = 0;
    if (S->pb.t_end > 0.0 && S->info.t + dt >= S->pb.t_end) {
      dt = S->pb.t_end - S->info.t;
      last = 1;
    }
    /* moment update c(lambda_l, lambda_c, lambda_r), eq:momentIterationFunction
       in the quadrature form eq:momentUpQuadrature */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < S->cells; ++c) {
      if (S->pb.flux == ORC_FLUX_SG_ANALYTIC) {
        /* App. A, eq:numFluxAnalytic on the duals of the cell and its two
           neighbours (outflow: the cell itself, periodic: wrap) */
        int N = S->N, nx = S->pb.nx;
        int cw = c - 1, ce = c + 1;
        if (cw < 0) cw = S->pb.bc[0] == ORC_BC_PERIODIC ? nx - 1 : c;
        if (ce >= nx) ce = S->pb.bc[1] == ORC_BC_PERIODIC ? 0 : c;
        const double *lw = S->lam + (size_t)cw * n, *lc = S->lam + (size_t)c * n,
                     *le = S->lam + (size_t)ce * n;
        int Nn = S->pb.adapt ? orc_num_basis(S->pb.p, S->deg_next[c]) : S->Nc[c];
        double visc = S->dx / (2.0 * dt);
        for (int i = 0; i < N; ++i) {
          double Fw = 0.0, Fc = 0.0, Fe = 0.0;
          for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
              double C = S->Ctp[((size_t)i * N + a) * N + b];
              Fw += 0.5 * C * lw[a] * lw[b];
              Fc += 0.5 * C * lc[a] * lc[b];
              Fe += 0.5 * C * le[a] * le[b];
            }
          double Gr = 0.5 * (Fc + Fe) - visc * (le[i] - lc[i]);
          double Gl = 0.5 * (Fw + Fc) - visc * (lc[i] - lw[i]);
          S->unew[(size_t)c * n + i] = i < Nn ? lc[i] - dt / S->dx * (Gr - Gl) : 0.0;
        }
        continue;
      }
      int ix = c % S->pb.nx, iy = c / S->pb.nx;
      const double *uc = S->nodal + (size_t)c * Q * m;
      const double *uw = neighbour(S, ix, iy, 0), *ue = neighbour(S, ix, iy, 1);
      const double *us = S->dim == 2 ? neighbour(S, ix, iy, 2) : NULL;
      const double *un = S->dim == 2 ? neighbour(S, ix, iy, 3) : NULL;
      double *acc = (double *)malloc(sizeof(double) * Q * m);
      for (int q = 0; q < Q; ++q) {
        double gl[ORC_MAXM], gr[ORC_MAXM];
        num_flux(S, 0, uc + q * m, ue + q * m, dt, gr);
        num_flux(S, 0, uw + q * m, uc + q * m, dt, gl);
        for (int a = 0; a < m; ++a)
          acc[q * m + a] = uc[q * m + a] - dt / S->dx * (gr[a] - gl[a]);
        if (S->dim == 2) {
          num_flux(S, 1, uc + q * m, un + q * m, dt, gr);
          num_flux(S, 1, us + q * m, uc + q * m, dt, gl);
          for (int a = 0; a < m; ++a) acc[q * m + a] -= dt / S->dy * (gr[a] - gl[a]);
        }
      }
      /* adaptive: eq:adaptiveFVUpdate, the projection on the new level */
      int Nn = S->pb.adapt ? orc_num_basis(S->pb.p, S->deg_next[c]) : S->Nc[c];
      project(S, Nn, acc, S->unew + (size_t)c * n);
      free(acc);
    }
    /* steady residual eq:residualSteady, fixed summation order */
    double res = 0.0;
    for (int c = 0; c < S->cells; ++c) {
      double s2 = 0.0;
      for (int k = 0; k < n; ++k) {
        double dlt = S->unew[(size_t)c * n + k] - S->uhat[(size_t)c * n + k];
        s2 += dlt * dlt;
      }
      res += S->vol * sqrt(s2);
    }
    for (size_t k = 0; k < (size_t)S->cells * n; ++k)
      if (!isfinite(S->unew[k])) { st |= ORC_ST_NONFINITE; break; }
    double *tmp = S->uhat;
    S->uhat = S->unew;
    S->unew = tmp;
    /* adaptive: the dual of the next step keeps the modes of the new level
       (padded with zeros when the level rises) */
    if (S->pb.adapt)
      for (int c = 0; c < S->cells; ++c) {
        int Nn = orc_num_basis(S->pb.p, S->deg_next[c]);
        for (int a = 0; a < m; ++a)
          for (int i = Nn; i < S->N; ++i) S->lam[(size_t)c * n + a * S->N + i] = 0.0;
        S->Nc[c] = Nn;
        S->deg[c] = S->deg_next[c];
      }
    S->info.t = last ? S->pb.t_end : S->info.t + dt;
    S->info.dt = dt;
    S->info.amax = S->dim == 2 ? (ax > ay ? ax : ay) : ax;
    S->info.residual = res;
    S->info.steps += 1;
    S->info.newton_iters += its;
    S->info.cell_updates += S->cells;
    if (maxit > S->info.max_iters) S->info.max_iters = maxit;
    S->info.status |= st;
    /* steady stop (eq:residualSteady); with retardation only in the last
       stage, and otherwise the stage advances at its tolerance */
    int final_stage = S->pb.n_retard == 0 || S->info.retard_stage == S->pb.n_retard - 1;
    if (last || (S->pb.steady_eps > 0.0 && final_stage && res <= S->pb.steady_eps) ||
        S->info.status)
      S->info.done = 1;
    else if (!final_stage && res <= S->pb.retard_eps[S->info.retard_stage])
      S->info.retard_stage += 1;
  }
  if (info) *info = S->info;
  return S->info.status;
}

void orc_get_info(const orc_state *S, orc_info *info) { *info = S->info; }

void orc_get_moments(const orc_state *S, double *out)
{
  memcpy(out, S->uhat, sizeof(double) * S->cells * S->n);
}

void orc_set_moments(orc_state *S, const double *in)
{
  memcpy(S->uhat, in, sizeof(double) * S->cells * S->n);
}

void orc_get_dual(const orc_state *S, double *out)
{
  memcpy(out, S->lam, sizeof(double) * S->cells * S->n);
}

void orc_set_dual(orc_state *S, const double *in)
{
  memcpy(S->lam, in, sizeof(double) * S->cells * S->n);
}

void orc_get_iters(const orc_state *S, int *out) { memcpy(out, S->iters, sizeof(int) * S->cells); }

void orc_get_degrees(const orc_state *S, signed char *out)
{
  for (int c = 0; c < S->cells; ++c) out[c] = (signed char)S->deg[c];
}

int orc_get_nodal(const orc_state *S, double *out)
{
  int ok = 1;
  for (int c = 0; c < S->cells; ++c)
    ok &= cell_nodal(S, S->Nc[c], S->lam + (size_t)c * S->n, out + (size_t)c * S->Q * S->m);
  return ok;
}

void orc_tables(const orc_state *S, double *nodes, double *w, double *Phi)
{
  if (nodes) memcpy(nodes, S->nodes, sizeof(double) * S->Q * S->pb.p);
  if (w) memcpy(w, S->w, sizeof(double) * S->Q);
  if (Phi) memcpy(Phi, S->Phi, sizeof(double) * S->Q * S->N);
}

/* L, grad L ([m][N]) and H ([mN][mN], variable-major (a,i)) at lam */
int orc_dual_cost(const orc_state *S, const double *lam, const double *uhat, double *L,
                  double *grad, double *H)
{
  scratch_t w = scratch_alloc(S);
  int ok = eval_nodes(S, S->N, lam, w.u, w.J, w.ss);
  if (ok) {
    *L = dual_cost_from_nodes(S, S->N, lam, uhat, w.ss);
    dual_gradient(S, S->N, w.u, uhat, grad);
    if (H) dual_hessian(S, S->N, w.J, H);
  }
  scratch_free(&w);
  return ok;
}

int orc_dual_solve(const orc_state *S, const double *uhat, double *lam, int one_shot, int *iters)
{
  scratch_t w = scratch_alloc(S);
  int st = dual_newton(S, S->N, uhat, lam, one_shot, iters, &w);
  scratch_free(&w);
  return st;
}

int orc_moments_of_dual(const orc_state *S, const double *lam, double *uhat)
{
  double *nod = (double *)malloc(sizeof(double) * S->Q * S->m);
  int ok = cell_nodal(S, S->N, lam, nod);
  project(S, S->N, nod, uhat);
  free(nod);
  return ok;
}
