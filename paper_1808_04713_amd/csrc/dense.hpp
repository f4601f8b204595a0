// Small dense linear algebra for host-side setup (n up to a few hundred):
// LU with partial pivoting, Cholesky, symmetric Jacobi eigensolver and a
// complex Hessenberg-QR eigensolver.  Column-major storage throughout.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

namespace hdp {

using cd = std::complex<double>;

template <class T>
struct Mat {
  int r = 0, c = 0;
  std::vector<T> a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a(size_t(r_) * c_, T(0)) {}
  T& operator()(int i, int j) { return a[size_t(j) * r + i]; }
  const T& operator()(int i, int j) const { return a[size_t(j) * r + i]; }
  static Mat eye(int n) {
    Mat m(n, n);
    for (int i = 0; i < n; ++i) m(i, i) = T(1);
    return m;
  }
};
using MatD = Mat<double>;
using MatC = Mat<cd>;

template <class A, class B>
auto matmul(const Mat<A>& x, const Mat<B>& y) {
  using R = decltype(A() * B());
  if (x.c != y.r) throw std::runtime_error("matmul shape");
  Mat<R> z(x.r, y.c);
  for (int j = 0; j < y.c; ++j)
    for (int k = 0; k < x.c; ++k) {
      R b = R(y(k, j));
      if (b == R(0)) continue;
      for (int i = 0; i < x.r; ++i) z(i, j) += R(x(i, k)) * b;
    }
  return z;
}

template <class T>
Mat<T> transpose(const Mat<T>& x) {
  Mat<T> y(x.c, x.r);
  for (int j = 0; j < x.c; ++j)
    for (int i = 0; i < x.r; ++i) y(j, i) = x(i, j);
  return y;
}

inline MatC to_complex(const MatD& x) {
  MatC y(x.r, x.c);
  for (size_t i = 0; i < x.a.size(); ++i) y.a[i] = x.a[i];
  return y;
}

// In-place LU with partial pivoting; returns false if a pivot is exactly zero.
template <class T>
bool lu_factor(Mat<T>& A, std::vector<int>& piv) {
  int n = A.r;
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(A(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > best) { best = std::abs(A(i, k)); p = i; }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
    T inv = T(1) / A(k, k);
    for (int i = k + 1; i < n; ++i) A(i, k) *= inv;
    for (int j = k + 1; j < n; ++j) {
      T f = A(k, j);
      if (f == T(0)) continue;
      for (int i = k + 1; i < n; ++i) A(i, j) -= A(i, k) * f;
    }
  }
  return true;
}

template <class T>
void lu_solve(const Mat<T>& LU, const std::vector<int>& piv, Mat<T>& B) {
  int n = LU.r;
  for (int j = 0; j < B.c; ++j) {
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(B(k, j), B(piv[k], j));
    for (int k = 0; k < n; ++k) {
      T b = B(k, j);
      for (int i = k + 1; i < n; ++i) B(i, j) -= LU(i, k) * b;
    }
    for (int k = n - 1; k >= 0; --k) {
      B(k, j) /= LU(k, k);
      T b = B(k, j);
      for (int i = 0; i < k; ++i) B(i, j) -= LU(i, k) * b;
    }
  }
}

template <class T>
Mat<T> solve(Mat<T> A, Mat<T> B) {
  std::vector<int> piv;
  if (!lu_factor(A, piv)) throw std::runtime_error("singular matrix");
  lu_solve(A, piv, B);
  return B;
}

template <class T>
Mat<T> inverse(const Mat<T>& A) { return solve(A, Mat<T>::eye(A.r)); }

// Cholesky A = L L^T of a symmetric positive definite matrix (lower factor).
inline MatD cholesky(const MatD& A) {
  int n = A.r;
  MatD L(n, n);
  for (int j = 0; j < n; ++j) {
    double s = A(j, j);
    for (int k = 0; k < j; ++k) s -= L(j, k) * L(j, k);
    if (s <= 0) throw std::runtime_error("cholesky: not positive definite");
    L(j, j) = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A(i, j);
      for (int k = 0; k < j; ++k) t -= L(i, k) * L(j, k);
      L(i, j) = t / L(j, j);
    }
  }
  return L;
}

// Cyclic Jacobi for a real symmetric matrix: A = V diag(w) V^T.
inline void jacobi_eig(MatD A, std::vector<double>& w, MatD& V) {
  int n = A.r;
  V = MatD::eye(n);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        tot += A(i, j) * A(i, j);
        if (i != j) off += A(i, j) * A(i, j);
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A(p, q);
        if (std::abs(apq) < 1e-300) continue;
        double theta = (A(q, q) - A(p, p)) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A(k, p), akq = A(k, q);
          A(k, p) = c * akp - s * akq;
          A(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A(p, k), aqk = A(q, k);
          A(p, k) = c * apk - s * aqk;
          A(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V(k, p), vkq = V(k, q);
          V(k, p) = c * vkp - s * vkq;
          V(k, q) = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

// Eigen-decomposition of a general complex matrix by Householder reduction to
// Hessenberg form and single-shift QR (Wilkinson shifts) with accumulated
// unitary transforms; eigenvectors by back substitution on the Schur form.
// Returns eigenvalues lam and eigenvectors as the columns of X (unnormalised).
inline void complex_eig(MatC A, std::vector<cd>& lam, MatC& X) {
  int n = A.r;
  MatC Q = MatC::eye(n);
  // Hessenberg reduction
  for (int k = 0; k < n - 2; ++k) {
    double alpha = 0;
    for (int i = k + 1; i < n; ++i) alpha += std::norm(A(i, k));
    alpha = std::sqrt(alpha);
    if (alpha == 0) continue;
    std::vector<cd> v(n, 0);
    cd x0 = A(k + 1, k);
    cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1);
    v[k + 1] = x0 + ph * alpha;
    for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
    double vn = 0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0) continue;
    // A = (I - 2 v v^H / vn) A (I - 2 v v^H / vn)
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * A(i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) A(i, j) -= v[i] * s;
    }
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) A(i, j) -= s * std::conj(v[j]);
    }
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int j = k + 1; j < n; ++j) s += Q(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) Q(i, j) -= s * std::conj(v[j]);
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 2; i < n; ++i) A(i, j) = 0;
  // shifted QR on the active window [lo, hi]
  int hi = n - 1, iter = 0;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      double s = std::abs(A(lo - 1, lo - 1)) + std::abs(A(lo, lo));
      if (s == 0) s = 1;
      if (std::abs(A(lo, lo - 1)) < 1e-16 * s) { A(lo, lo - 1) = 0; break; }
      --lo;
    }
    if (lo == hi) { --hi; iter = 0; continue; }
    if (++iter > 300) throw std::runtime_error("complex_eig: QR did not converge");
    // Wilkinson shift from the trailing 2x2 block
    cd a = A(hi - 1, hi - 1), b = A(hi - 1, hi), c = A(hi, hi - 1), d = A(hi, hi);
    cd tr = a + d, det = a * d - b * c;
    cd disc = std::sqrt(tr * tr / 4.0 - det);
    cd m1 = tr / 2.0 + disc, m2 = tr / 2.0 - disc;
    cd mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    if (iter % 11 == 10) mu = d + std::abs(A(hi, hi - 1));  // exceptional shift
    // implicit single-shift QR sweep via Givens rotations
    cd x = A(lo, lo) - mu, y = A(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cd cs = r > 0 ? x / r : cd(1), sn = r > 0 ? y / r : cd(0);
      // rotation G = [conj(cs) conj(sn); -sn cs] on rows k, k+1
      int j0 = std::max(lo, k - 1);
      for (int j = j0; j < n; ++j) {
        cd t1 = A(k, j), t2 = A(k + 1, j);
        A(k, j) = std::conj(cs) * t1 + std::conj(sn) * t2;
        A(k + 1, j) = -sn * t1 + cs * t2;
      }
      int i1 = std::min(hi, k + 2);
      for (int i = 0; i <= i1; ++i) {
        cd t1 = A(i, k), t2 = A(i, k + 1);
        A(i, k) = t1 * cs + t2 * sn;
        A(i, k + 1) = -t1 * std::conj(sn) + t2 * std::conj(cs);
      }
      for (int i = 0; i < n; ++i) {
        cd t1 = Q(i, k), t2 = Q(i, k + 1);
        Q(i, k) = t1 * cs + t2 * sn;
        Q(i, k + 1) = -t1 * std::conj(sn) + t2 * std::conj(cs);
      }
      if (k + 1 < hi) {
        x = A(k + 1, k);
        y = A(k + 2, k);
      }
    }
  }
  // eigenvectors of the upper-triangular Schur factor T = A
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A(i, i);
  MatC Y(n, n);
  double scale = 0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(A(i, i)));
  double small = std::max(scale, 1.0) * 1e-15;
  for (int k = 0; k < n; ++k) {
    Y(k, k) = 1;
    for (int i = k - 1; i >= 0; --i) {
      cd s = 0;
      for (int j = i + 1; j <= k; ++j) s += A(i, j) * Y(j, k);
      cd den = A(i, i) - lam[k];
      if (std::abs(den) < small) den = small;
      Y(i, k) = -s / den;
    }
  }
  X = matmul(Q, Y);
}

}  // namespace hdp
