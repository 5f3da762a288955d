// Host-side construction of the quadrature rule and the gPC basis table.
//
// Gauss-Legendre nodes (Sec. 3.1, quadrature <h>_Q with the uniform density
// folded into the weights) and the orthonormal total-degree Legendre basis
// (Sec. 2, eq:numberBasisFcts); the table A_{ki} = phi_i(xi_k) of App. A is
// built once per problem and uploaded.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

namespace ipm {

inline int binom_basis(int p, int degree) {
  long long r = 1;
  for (int k = 1; k <= p; ++k) r = r * (degree + k) / k;
  return static_cast<int>(r);
}

// Three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; returns
// P_n(x) and P_{n-1}(x).
inline void legendre_pair(int n, double x, double& pn, double& pnm1) {
  double a = 1.0, b = x;
  if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
    a = b;
    b = c;
  }
  pn = b;
  pnm1 = a;
}

// n-point Gauss-Legendre rule on [-1, 1]: Tricomi's estimate of the k-th
// root, refined by Newton's method on P_n; weights 2 / ((1-x^2) P_n'(x)^2)
// with P_n' = n (x P_n - P_{n-1}) / (x^2 - 1).  Nodes ascending.
inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 1; k <= n; ++k) {
    const double th = pi * (4.0 * k - 1.0) / (4.0 * n + 2.0);
    double z = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * std::cos(th);
    double pn = 0, pm = 0;
    for (int it = 0; it < 64; ++it) {
      legendre_pair(n, z, pn, pm);
      const double d = n * (z * pn - pm) / (z * z - 1.0);
      const double step = pn / d;
      z -= step;
      if (std::fabs(step) < 5e-17) break;
    }
    legendre_pair(n, z, pn, pm);
    const double d = n * (z * pn - pm) / (z * z - 1.0);
    x[n - k] = z;
    w[n - k] = 2.0 / ((1.0 - z * z) * d * d);
  }
}

// Tensor rule for xi ~ U(-1,1)^p.  Node q has digits (q_1 .. q_p) in base
// qpd with q_1 most significant; weight prod_k w_{q_k} / 2 (sums to one).
inline int tensor_rule(int p, int qpd, std::vector<double>& nodes, std::vector<double>& wts) {
  std::vector<double> x, w;
  gauss_legendre(qpd, x, w);
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= qpd;
  nodes.assign(static_cast<size_t>(Q) * p, 0.0);
  wts.assign(Q, 1.0);
  for (int q = 0; q < Q; ++q) {
    int r = q;
    for (int k = p - 1; k >= 0; --k) {
      const int d = r % qpd;
      r /= qpd;
      nodes[static_cast<size_t>(q) * p + k] = x[d];
      wts[q] *= 0.5 * w[d];
    }
  }
  return Q;
}

// Multi-indices with |i| <= degree, graded: total degree ascending, then the
// first exponent descending (lexicographically descending within a degree).
// Every lower-degree set is a prefix, which per-cell degrees rely on.
inline std::vector<int> graded_indices(int p, int degree) {
  std::vector<int> out;
  std::vector<int> e(p, 0);
  for (int d = 0; d <= degree; ++d) {
    // odometer over compositions of d into p parts, first part descending
    e.assign(p, 0);
    e[0] = d;
    while (true) {
      out.insert(out.end(), e.begin(), e.end());
      // next composition in lexicographically descending order
      int k = p - 2;
      while (k >= 0 && e[k] == 0) --k;
      if (k < 0) break;
      e[k] -= 1;
      int rest = 0;
      for (int j = k + 1; j < p; ++j) rest += e[j];
      for (int j = k + 1; j < p; ++j) e[j] = 0;
      e[k + 1] = rest + 1;
    }
  }
  return out;
}

// Phi[q][i] = prod_k sqrt(2 i_k + 1) P_{i_k}(xi_{q,k}).
inline std::vector<double> basis_table(int p, int degree, int Q, const std::vector<double>& nodes) {
  const int N = binom_basis(p, degree);
  const std::vector<int> idx = graded_indices(p, degree);
  std::vector<double> Phi(static_cast<size_t>(Q) * N);
  for (int q = 0; q < Q; ++q)
    for (int i = 0; i < N; ++i) {
      double v = 1.0;
      for (int k = 0; k < p; ++k) {
        const int e = idx[static_cast<size_t>(i) * p + k];
        double pn, pm;
        legendre_pair(e, nodes[static_cast<size_t>(q) * p + k], pn, pm);
        v *= std::sqrt(2.0 * e + 1.0) * pn;
      }
      Phi[static_cast<size_t>(q) * N + i] = v;
    }
  return Phi;
}

}  // namespace ipm
