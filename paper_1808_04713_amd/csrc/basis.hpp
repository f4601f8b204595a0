// One-dimensional spectral toolkit (paper Sec. 2.1.1): orthonormal Legendre
// polynomials, the integrated-Legendre basis N = S p, its stiffness and mass
// matrices, the vertex ("interpolatory") basis N~ = B N, quadrature rules.
#pragma once
#include <cmath>
#include <vector>

#include "dense.hpp"

namespace hdp {

// p_0..p_{n-1} at x by the three-term recurrence (eq. recurrence_relation).
inline void legendre_p(int n, double x, double* p) {
  p[0] = 1.0 / std::sqrt(2.0);
  if (n > 1) p[1] = std::sqrt(1.5) * x;
  for (int k = 2; k < n; ++k)
    p[k] = std::sqrt((2.0 * k + 1) * (2.0 * k - 1)) / k * x * p[k - 1] -
           (k - 1.0) / k * std::sqrt((2.0 * k + 1) / (2.0 * k - 3)) * p[k - 2];
}

// Gauss-Legendre nodes and weights on [-1,1] by Newton iteration on P_q.
inline void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = t;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = t; p0 = 1; }
      dp = q * (t * p1 - p0) / (t * t - 1);
      double dt = p1 / dp;
      t -= dt;
      if (std::abs(dt) < 1e-16) break;
    }
    double p0 = 1, p1 = t;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = t; p0 = 1; }
    dp = q * (t * p1 - p0) / (t * t - 1);
    x[q - 1 - i] = t;
    w[q - 1 - i] = 2.0 / ((1 - t * t) * dp * dp);
  }
}

// Gauss-Lobatto-Legendre nodes for degree p (p+1 nodes): -1, +1 and the
// roots of P_p', by Newton iteration from Chebyshev-Lobatto starting points.
inline std::vector<double> gll_nodes(int n) {
  int p = n - 1;
  std::vector<double> t(n);
  for (int i = 0; i < n; ++i) t[i] = -std::cos(M_PI * i / p);
  for (int i = 1; i < p; ++i) {
    double x = t[i];
    for (int it = 0; it < 100; ++it) {
      // P_p, P_p', P_p'' by recurrence
      double p0 = 1, p1 = x;
      for (int k = 2; k <= p; ++k) {
        double p2 = ((2.0 * k - 1) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double P = p1, Pm = p0;
      double d1 = p * (x * P - Pm) / (x * x - 1);
      double d2 = (2 * x * d1 - p * (p + 1.0) * P) / (1 - x * x);
      double dx = d1 / d2;
      x -= dx;
      if (std::abs(dx) < 1e-16) break;
    }
    t[i] = x;
  }
  t[0] = -1;
  t[p] = 1;
  return t;
}

// S of eq. (define_basis_functions): N = S p.
inline MatD basis_S(int n) {
  MatD S(n, n);
  std::vector<double> g(n, 1.0);
  for (int i = 2; i <= n; ++i) g[i - 1] = 1.0 / std::sqrt((2.0 * i - 1) * (2.0 * i - 3));
  for (int i = 0; i < n; ++i) S(i, i) = g[i];
  for (int i = 2; i < n; ++i) S(i, i - 2) = -g[i - 1];
  return S;
}

// Integrated-Legendre basis values N_k(x), k < n.
inline void basis_N(int n, double x, double* N) {
  std::vector<double> p(n);
  legendre_p(n, x, p.data());
  MatD S = basis_S(n);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < n; ++j) s += S(i, j) * p[j];
    N[i] = s;
  }
}

// Vertex basis N~ = B N: N~_0 = (1+x)/2, N~_1 = (1-x)/2, N~_k = N_k for k >= 2.
inline void vertex_basis(int n, double x, double* Nt) {
  basis_N(n, x, Nt);
  double a = Nt[0], b = n > 1 ? Nt[1] : 0.0;
  Nt[0] = (a + b) / std::sqrt(2.0);
  if (n > 1) Nt[1] = (a - b) / std::sqrt(2.0);
}

// Derivative of the vertex basis: d/dx N = S_DL p, then B.
inline void vertex_basis_dx(int n, double x, double* dNt) {
  std::vector<double> p(n);
  legendre_p(n, x, p.data());
  std::vector<double> d(n, 0.0);
  for (int i = 1; i < n; ++i) d[i] = p[i - 1];
  dNt[0] = (d[0] + (n > 1 ? d[1] : 0.0)) / std::sqrt(2.0);
  if (n > 1) dNt[1] = (d[0] - d[1]) / std::sqrt(2.0);
  for (int i = 2; i < n; ++i) dNt[i] = d[i];
}

// 1-D stiffness K^ = S_DL S_DL^T and mass M^ = S S^T, transformed to the
// vertex basis (B K^ B, B M^ B).
inline MatD stiffness_vertex(int n) {
  MatD K(n, n);
  for (int i = 1; i < n; ++i) K(i, i) = 1.0;
  // B K^ B with K^ = diag(0,1,..): only the top 2x2 block changes
  if (n > 1) {
    K(0, 0) = 0.5; K(1, 1) = 0.5; K(0, 1) = -0.5; K(1, 0) = -0.5;
  }
  return K;
}

inline MatD mass_vertex(int n) {
  MatD S = basis_S(n);
  MatD M = matmul(S, transpose(S));
  MatD B = MatD::eye(n);
  if (n > 1) {
    double r = 1.0 / std::sqrt(2.0);
    B(0, 0) = r; B(0, 1) = r; B(1, 0) = r; B(1, 1) = -r;
  }
  return matmul(matmul(B, M), B);
}

// Dispersion rule of Sec. 2.3.4: smallest integer l > (kh + (kh)^(1/3) - 1)/2, l >= 1.
inline int dispersion_l(double k, double h) {
  double x = 0.5 * (k * h + std::cbrt(k * h) - 1.0);
  int l = int(std::floor(x)) + 1;
  return l < 1 ? 1 : l;
}

}  // namespace hdp
