// Device building blocks shared by the IPM kernels: wave-level LDS
// ordering, the entropy closures u_s = (grad s)^-1 with their Jacobians and
// Legendre duals (Sec. 2 eq:ansatz, Sec. 3.1; App. B), physical fluxes and
// the deterministic numerical fluxes of the kinetic flux (Sec. 3.1-3.2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipm {

enum { kBurgers1D = 0, kEuler1D = 1, kEuler2D = 2 };
enum { kEntQuadratic = 0, kEntLogBarrier = 1, kEntEuler = 2 };
// kFluxSgAnalytic: App. A, eq:numFluxAnalytic (Burgers, quadratic entropy)
enum { kFluxLF = 0, kFluxRusanov = 1, kFluxSgAnalytic = 2 };
enum { kBcOutflow = 0, kBcPeriodic = 1, kBcDirichlet = 2 };

// status bits kept per problem on the device
enum : unsigned {
  kStNewton = 1u,
  kStRealizability = 2u,
  kStNonfinite = 4u,
  kStPivot = 8u,  // a non-positive pivot in the SPD elimination
  kStLineSearch = 16u,
};

struct ClosureParams {
  int entropy;
  int g75;  // gamma = 7/5: the Euler closure's power of beta in closed form
  double gamma, um, up;
  double log_range;  // ln(u_plus - u_minus), log-barrier constant of s_*
  double r1mg;       // 1 / (1 - gamma): the Euler closure multiplies by it
};

// Orders LDS traffic between the lanes of one wavefront (no s_barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M>
struct Packed {
  static constexpr int NJ = M * (M + 1) / 2;
  // index of (a, b), a <= b, in row-major upper-triangle packing
  __host__ __device__ static constexpr int idx(int a, int b) {
    return a <= b ? a * M - a * (a - 1) / 2 + (b - a) : b * M - b * (b - 1) / 2 + (a - b);
  }
};

// Ansatz at one node.  Returns false outside the closure's domain.
// J is the packed symmetric Jacobian grad u_s (upper triangle).
template <int M>
__device__ __forceinline__ bool closure(const ClosureParams& cp, const double* L, double* u,
                                        double* J, double& sstar) {
  if (cp.entropy == kEntQuadratic) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      u[a] = L[a];
      s += L[a] * L[a];
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = a; b < M; ++b) J[Packed<M>::idx(a, b)] = (a == b) ? 1.0 : 0.0;
    sstar = 0.5 * s;
    if constexpr (M >= 3) {
      // gas dynamics: a stochastic-Galerkin state with a non-positive
      // density or pressure at a node has no physical flux (SG's failure)
      double mm = 0.0;
#pragma unroll
      for (int k = 1; k < M - 1; ++k) mm += u[k] * u[k];
      if (!(u[0] > 0.0)) return false;
      if (!((cp.gamma - 1.0) * (u[M - 1] - 0.5 * mm / u[0]) > 0.0)) return false;
    }
    return true;
  }
  if (M == 1 && cp.entropy == kEntLogBarrier) {
    // u_s = u_- + D sigma(L), u_s' = D sigma (1 - sigma),
    // s_* = u_- L + D softplus(L) - D ln D, with D = u_+ - u_-
    const double D = cp.up - cp.um;
    const double x = L[0];
    const double e = exp(-fabs(x));
    const double inv = 1.0 / (1.0 + e);
    const double sig = x >= 0.0 ? inv : e * inv;
    const double oms = x >= 0.0 ? e * inv : inv;
    u[0] = cp.um + D * sig;
    J[0] = D * sig * oms;
    sstar = cp.um * x + D * (fmax(x, 0.0) + log1p(e)) - D * cp.log_range;
    return true;
  }
  if (M >= 3) {
    // Euler entropy (App. B): with beta = -L_E, v = L_m / beta, e = 1/beta,
    // ln rho = (ln beta - |L_m|^2 / (2 beta) + gamma - L_rho) / (1 - gamma);
    // grad u_s = rho/(gamma-1) w w^T + rho e (sum_k a_k a_k^T + e eE eE^T)
    // with w = (1, v, h), a_k = (0, unit_k, v_k), h = |v|^2/2 + e.
    constexpr int d = M - 2;
    const double beta = -L[M - 1];
    if (!(beta > 0.0)) return false;
    const double ib = 1.0 / beta;
    double v[2] = {0.0, 0.0};
    double vv = 0.0;
#pragma unroll
    for (int k = 0; k < d; ++k) {
      v[k] = L[1 + k] * ib;
      vv += v[k] * v[k];
    }
    // rho = beta^(1/(1-gamma)) exp((gamma - L_rho - |L_m|^2/(2 beta)) / (1-gamma));
    // for gamma = 7/5 the power is beta^(-5/2) = ib^2 sqrt(ib): a square
    // root instead of a logarithm
    const double rho = cp.g75 ? exp((cp.gamma - L[0] - 0.5 * beta * vv) * cp.r1mg) * (ib * ib * sqrt(ib))
                              : exp((log(beta) - 0.5 * beta * vv + cp.gamma - L[0]) * cp.r1mg);
    const double h = 0.5 * vv + ib;
    u[0] = rho;
#pragma unroll
    for (int k = 0; k < d; ++k) u[1 + k] = rho * v[k];
    u[M - 1] = rho * h;
    const double c1 = rho / (cp.gamma - 1.0);
    const double c2 = rho * ib;
    double w[M];
    w[0] = 1.0;
#pragma unroll
    for (int k = 0; k < d; ++k) w[1 + k] = v[k];
    w[M - 1] = h;
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = a; b < M; ++b) {
        double s = c1 * w[a] * w[b];
        const bool am = a >= 1 && a <= d, bm = b >= 1 && b <= d;
        if (am && bm && a == b) s += c2;
        if (am && b == M - 1) s += c2 * v[a - 1];
        if (a == M - 1 && b == M - 1) s += c2 * (vv + ib);
        J[Packed<M>::idx(a, b)] = s;
      }
    sstar = (cp.gamma - 1.0) * rho;
    return rho == rho && rho < 1e300;
  }
  return false;
}

// Entropy variables grad s(u) (initial dual state).  False if u lies outside
// the entropy's domain.
template <int M>
__device__ __forceinline__ bool entropy_gradient(const ClosureParams& cp, const double* u,
                                                 double* L) {
  if (cp.entropy == kEntQuadratic) {
#pragma unroll
    for (int a = 0; a < M; ++a) L[a] = u[a];
    return true;
  }
  if (M == 1 && cp.entropy == kEntLogBarrier) {
    if (!(u[0] > cp.um && u[0] < cp.up)) return false;
    L[0] = log((u[0] - cp.um) / (cp.up - u[0]));
    return true;
  }
  if (M >= 3) {
    constexpr int d = M - 2;
    const double rho = u[0];
    double mm = 0.0;
#pragma unroll
    for (int k = 0; k < d; ++k) mm += u[1 + k] * u[1 + k];
    const double eps = u[M - 1] - 0.5 * mm / rho;  // internal energy per volume
    if (!(rho > 0.0 && eps > 0.0)) return false;
    // ds/drho = gamma ln rho - ln eps - |m|^2/(2 rho eps) + gamma,
    // ds/dm = m / eps, ds/dE = -rho / eps
    L[0] = cp.gamma * log(rho) - log(eps) - 0.5 * mm / (rho * eps) + cp.gamma;
#pragma unroll
    for (int k = 0; k < d; ++k) L[1 + k] = u[1 + k] / eps;
    L[M - 1] = -rho / eps;
    return true;
  }
  return false;
}

// Physical flux in direction dir and the spectral radius of its Jacobian.
template <int M>
__device__ __forceinline__ void physical_flux(double gamma, int dir, const double* u, double* f,
                                              double& speed) {
  if (M == 1) {
    f[0] = 0.5 * u[0] * u[0];
    speed = fabs(u[0]);
    return;
  }
  constexpr int d = M - 2;
  const double rho = u[0];
  const double ir = 1.0 / rho;
  double vv = 0.0;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < d; ++k) {
    v[k] = u[1 + k] * ir;
    vv += v[k] * v[k];
  }
  const double E = u[M - 1];
  const double p = (gamma - 1.0) * (E - 0.5 * rho * vv);
  const double vn = v[dir];
  f[0] = rho * vn;
#pragma unroll
  for (int k = 0; k < d; ++k) f[1 + k] = u[1 + k] * vn + (k == dir ? p : 0.0);
  f[M - 1] = (E + p) * vn;
  speed = fabs(vn) + sqrt(gamma * p * ir);
}

// The quantities of a node state that its fluxes in every direction share
// (gas dynamics: 1/rho, velocity, pressure and sound speed), formed with the
// same operations as physical_flux, so fluxes and speeds built from them
// equal physical_flux's bit for bit with one division and one square root
// per state.
template <int M>
struct FluxState {
  double ir = 0.0, p = 0.0, a = 0.0;
  double v[2] = {0.0, 0.0};
};

template <int M>
__device__ __forceinline__ FluxState<M> flux_state(double gamma, const double* u) {
  FluxState<M> s;
  if (M == 1) return s;
  constexpr int d = M - 2;
  const double rho = u[0];
  s.ir = 1.0 / rho;
  double vv = 0.0;
#pragma unroll
  for (int k = 0; k < d; ++k) {
    s.v[k] = u[1 + k] * s.ir;
    vv += s.v[k] * s.v[k];
  }
  s.p = (gamma - 1.0) * (u[M - 1] - 0.5 * rho * vv);
  s.a = sqrt(gamma * s.p * s.ir);
  return s;
}

// physical_flux from a state's shared quantities
template <int M>
__device__ __forceinline__ void state_flux(const FluxState<M>& s, int dir, const double* u,
                                           double* f, double& speed) {
  if (M == 1) {
    f[0] = 0.5 * u[0] * u[0];
    speed = fabs(u[0]);
    return;
  }
  constexpr int d = M - 2;
  const double vn = s.v[dir];
  f[0] = u[0] * vn;
#pragma unroll
  for (int k = 0; k < d; ++k) f[1 + k] = u[1 + k] * vn + (k == dir ? s.p : 0.0);
  f[M - 1] = (u[M - 1] + s.p) * vn;
  speed = fabs(vn) + s.a;
}

// Wave speeds of one node state: sx (x-direction) and sy (y, 2D only).
template <int M>
__device__ __forceinline__ void wave_speeds(double gamma, int dim, const double* u, double& sx,
                                            double& sy) {
  double f[M];
  physical_flux<M>(gamma, 0, u, f, sx);
  sy = 0.0;
  if (dim == 2) physical_flux<M>(gamma, 1, u, f, sy);
}

// Deterministic numerical flux: Lax-Friedrichs g = (f_l + f_r)/2 -
// h/(2 dt) (u_r - u_l) or Rusanov with max(a_l, a_r)/2 as the viscosity.
template <int M>
__device__ __forceinline__ void numerical_flux(int kind, double gamma, int dir, const double* ul,
                                               const double* ur, double lf_visc, double* g) {
  double fl[M], fr[M], al, ar;
  physical_flux<M>(gamma, dir, ul, fl, al);
  physical_flux<M>(gamma, dir, ur, fr, ar);
  const double visc = kind == kFluxLF ? lf_visc : 0.5 * fmax(al, ar);
#pragma unroll
  for (int a = 0; a < M; ++a) g[a] = 0.5 * (fl[a] + fr[a]) - visc * (ur[a] - ul[a]);
}

// numerical_flux from the two states' shared quantities
template <int M>
__device__ __forceinline__ void numerical_flux_s(int kind, int dir, const double* ul,
                                                 const FluxState<M>& sl, const double* ur,
                                                 const FluxState<M>& sr, double lf_visc,
                                                 double* g) {
  double fl[M], fr[M], al, ar;
  state_flux<M>(sl, dir, ul, fl, al);
  state_flux<M>(sr, dir, ur, fr, ar);
  const double visc = kind == kFluxLF ? lf_visc : 0.5 * fmax(al, ar);
#pragma unroll
  for (int a = 0; a < M; ++a) g[a] = 0.5 * (fl[a] + fr[a]) - visc * (ur[a] - ul[a]);
}

// Non-negative doubles compare like their bit patterns (NaN above +inf).
__device__ __forceinline__ unsigned long long speed_bits(double s) {
  return static_cast<unsigned long long>(__double_as_longlong(s));
}

}  // namespace ipm
