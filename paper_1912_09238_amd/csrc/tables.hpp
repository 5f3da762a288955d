// Host-side construction of the quadrature rule and the gPC basis table.
//
// Gauss-Legendre nodes (Sec. 3.1, quadrature <h>_Q with the uniform density
// folded into the weights) and the orthonormal total-degree Legendre basis
// (Sec. 2, eq:numberBasisFcts); the table A_{ki} = phi_i(xi_k) of App. A is
// built once per problem and uploaded.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
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

// Clenshaw-Curtis rule of n points on [-1, 1] (the experiments of Sec. 7 use
// it for tensor and sparse grids): nodes cos(pi k / (n-1)) ascending, weights
// c_k / (n-1) * (1 - sum_{j=1}^{(n-1)/2} b_j cos(2 pi j k / (n-1)) / (4 j^2 - 1))
// with c_k = 1 at the end points (2 inside) and b_j = 1 for j = (n-1)/2 when
// n-1 is even (2 otherwise); n = 1 is the midpoint rule.  Weights sum to 2.
inline void clenshaw_curtis(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 2.0);
  if (n == 1) return;
  const double pi = 3.14159265358979323846;
  const int N = n - 1;
  for (int k = 0; k <= N; ++k) {
    double s = 0.0;
    for (int j = 1; j <= N / 2; ++j) {
      const double b = (2 * j == N) ? 1.0 : 2.0;
      s += b * std::cos(2.0 * pi * j * k / N) / (4.0 * j * j - 1.0);
    }
    const double c = (k == 0 || k == N) ? 1.0 : 2.0;
    x[N - k] = std::cos(pi * k / N);
    w[N - k] = c / N * (1.0 - s);
  }
  x[0] = -1.0;  // exact end points and centre
  x[N] = 1.0;
  if (N % 2 == 0) x[N / 2] = 0.0;
}

// Tensor rule of n points per dimension from a 1D rule (same node order and
// weight normalisation as tensor_rule).
inline int tensor_from_1d(int p, const std::vector<double>& x, const std::vector<double>& w,
                          std::vector<double>& nodes, std::vector<double>& wts) {
  const int n = static_cast<int>(x.size());
  int Q = 1;
  for (int k = 0; k < p; ++k) Q *= n;
  nodes.assign(static_cast<size_t>(Q) * p, 0.0);
  wts.assign(Q, 1.0);
  for (int q = 0; q < Q; ++q) {
    int r = q;
    for (int k = p - 1; k >= 0; --k) {
      const int d = r % n;
      r /= n;
      nodes[static_cast<size_t>(q) * p + k] = x[d];
      wts[q] *= 0.5 * w[d];
    }
  }
  return Q;
}

// Smolyak sparse grid of level L from the nested Clenshaw-Curtis rules with
// 1, 3, 5, 9, ..., 2^(l-1) + 1 points at levels l = 1, 2, 3, ...: the
// combination sum over l_1 + ... + l_p = s, s in [max(p, L+1), L+p], of
// (-1)^(L+p-s) binom(p-1, L+p-s) U_{l_1} x ... x U_{l_p}.  The rules are
// nested, so every node is a point of the finest grid (2^L + 1 points per
// dimension) and coinciding nodes are merged by their grid indices.  Nodes
// in ascending order of those indices; weights sum to one.
inline int cc_sparse_rule(int p, int L, std::vector<double>& nodes, std::vector<double>& wts) {
  const int fine = (1 << L) + 1;  // finest rule's points
  std::vector<double> xf, wf;
  clenshaw_curtis(fine, xf, wf);
  auto key_of = [&](const std::vector<int>& g) {
    long long k = 0;
    for (int d = 0; d < p; ++d) k = k * fine + g[d];
    return k;
  };
  std::vector<double> sum_w;
  std::vector<long long> sum_k;
  std::vector<int> l(p, 1);
  // enumerate l in [1, L+1]^p with sum in range (odometer)
  while (true) {
    int s = 0;
    for (int d = 0; d < p; ++d) s += l[d];
    if (s >= std::max(p, L + 1) && s <= L + p) {
      const int e = L + p - s;
      double coef = 1.0;
      for (int k = 1; k <= e; ++k) coef = coef * (p - k) / k;  // binom(p-1, e)
      if (e % 2) coef = -coef;
      // tensor product of the levels' rules
      std::vector<std::vector<double>> wl(p);
      std::vector<std::vector<int>> gl(p);
      for (int d = 0; d < p; ++d) {
        const int m = l[d] == 1 ? 1 : (1 << (l[d] - 1)) + 1;
        std::vector<double> xx, ww;
        clenshaw_curtis(m, xx, ww);
        wl[d] = ww;
        gl[d].resize(m);
        for (int k = 0; k < m; ++k) gl[d][k] = m == 1 ? (fine - 1) / 2 : k * ((fine - 1) / (m - 1));
      }
      std::vector<int> c(p, 0), g(p);
      while (true) {
        double w = coef;
        for (int d = 0; d < p; ++d) {
          w *= 0.5 * wl[d][c[d]];
          g[d] = gl[d][c[d]];
        }
        sum_k.push_back(key_of(g));
        sum_w.push_back(w);
        int d = p - 1;
        while (d >= 0 && ++c[d] == static_cast<int>(gl[d].size())) c[d--] = 0;
        if (d < 0) break;
      }
    }
    int d = p - 1;
    while (d >= 0 && ++l[d] > L + 1) l[d--] = 1;
    if (d < 0) break;
  }
  // merge by key
  std::vector<size_t> ord(sum_k.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
    return sum_k[a] != sum_k[b] ? sum_k[a] < sum_k[b] : a < b;
  });
  nodes.clear();
  wts.clear();
  for (size_t i = 0; i < ord.size();) {
    const long long k = sum_k[ord[i]];
    double w = 0.0;
    size_t j = i;
    for (; j < ord.size() && sum_k[ord[j]] == k; ++j) w += sum_w[ord[j]];
    long long r = k;
    std::vector<double> xn(p);
    for (int d = p - 1; d >= 0; --d) {
      xn[d] = xf[static_cast<size_t>(r % fine)];
      r /= fine;
    }
    nodes.insert(nodes.end(), xn.begin(), xn.end());
    wts.push_back(w);
    i = j;
  }
  return static_cast<int>(wts.size());
}

// Quadrature rules for xi ~ U(-1,1)^p selected by the problem: 0 tensor
// Gauss-Legendre with `param` points per dimension, 1 tensor Clenshaw-Curtis
// with `param` points per dimension, 2 Clenshaw-Curtis sparse grid of level
// `param`.  Returns Q (0 for an unknown rule).
inline int quadrature_rule(int rule, int p, int param, std::vector<double>& nodes,
                           std::vector<double>& wts) {
  if (rule == 0) return tensor_rule(p, param, nodes, wts);
  if (rule == 1) {
    std::vector<double> x, w;
    clenshaw_curtis(param, x, w);
    return tensor_from_1d(p, x, w, nodes, wts);
  }
  if (rule == 2) return cc_sparse_rule(p, param, nodes, wts);
  return 0;
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
