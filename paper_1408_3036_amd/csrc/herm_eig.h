// Eigen-decomposition of a small dense complex Hermitian matrix on the host
// (the per-band bases of the frequency recycling): Householder reduction to
// tridiagonal form, a diagonal phase that makes the off-diagonal real, then
// the implicit QL iteration with Wilkinson shifts on the real symmetric
// tridiagonal matrix, accumulating the eigenvectors.
#pragma once
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

namespace lgw {

// A: n x n row-major Hermitian (only its values are read; it is copied).
// On return w holds the eigenvalues in ascending order and V (n x n,
// row-major) the orthonormal eigenvectors as columns: A V[:, k] = w[k] V[:, k].
inline void herm_eig(int n, const std::complex<double>* A, std::vector<double>& w,
                     std::vector<std::complex<double>>& V) {
  using C = std::complex<double>;
  w.assign(n, 0.0);
  V.assign((size_t)n * n, C(0, 0));
  if (n <= 0) return;
  std::vector<C> a(A, A + (size_t)n * n);
  auto at = [&](int i, int j) -> C& { return a[(size_t)i * n + j]; };
  // Householder: Q^H A Q tridiagonal, Q = H_0 H_1 ... accumulated in V
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = C(1, 0);
  std::vector<C> v(n), p(n);
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(at(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const C x0 = at(k + 1, k);
    const C ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : C(1, 0);
    const C alpha = -ph * xn;                       // new sub-diagonal element
    for (int i = 0; i < n; ++i) v[i] = C(0, 0);
    for (int i = k + 1; i < n; ++i) v[i] = at(i, k);
    v[k + 1] -= alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // A <- H A H with H = I - 2 v v^H: p = A v, K = v^H p, q = 2 (p - K v),
    // A <- A - v q^H - q v^H  (over the rows and columns k..n-1)
    for (int i = k; i < n; ++i) {
      C s(0, 0);
      for (int j = k + 1; j < n; ++j) s += at(i, j) * v[j];
      p[i] = s;
    }
    C K(0, 0);
    for (int i = k + 1; i < n; ++i) K += std::conj(v[i]) * p[i];
    for (int i = k; i < n; ++i) p[i] = 2.0 * (p[i] - K * v[i]);
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j) at(i, j) -= v[i] * std::conj(p[j]) + p[i] * std::conj(v[j]);
    // Q <- Q H
    for (int r = 0; r < n; ++r) {
      C s(0, 0);
      for (int j = k + 1; j < n; ++j) s += V[(size_t)r * n + j] * v[j];
      for (int j = k + 1; j < n; ++j) V[(size_t)r * n + j] -= 2.0 * s * std::conj(v[j]);
    }
  }
  // T = D T_r D^H with a real non-negative sub-diagonal: phi_{k+1} = phi_k e_k / |e_k|
  std::vector<double> d(n), e(n, 0.0);
  std::vector<C> phi(n, C(1, 0));
  for (int k = 0; k < n; ++k) d[k] = at(k, k).real();
  for (int k = 0; k + 1 < n; ++k) {
    const C ek = at(k + 1, k);
    e[k] = std::abs(ek);
    phi[k + 1] = e[k] > 0.0 ? phi[k] * ek / e[k] : phi[k];
  }
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) V[(size_t)r * n + j] *= phi[j];
  // implicit QL on (d, e); e[i] couples i and i+1; Z accumulates the rotations
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (iter > 100) throw std::runtime_error("herm_eig: QL iteration did not converge");
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool deflated = false;
      for (int i = m - 1; i >= l; --i) {
        double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {   // underflow: the matrix splits at i + 1
          d[i + 1] -= pp;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          double* zk = &Z[(size_t)k * n];
          f = zk[i + 1];
          zk[i + 1] = s * zk[i] + c * f;
          zk[i] = c * zk[i] - s * f;
        }
      }
      if (deflated) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // ascending order; eigenvectors (Q D) Z
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && d[ord[j]] < d[ord[j - 1]]; --j) std::swap(ord[j], ord[j - 1]);
  std::vector<C> out((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int kk = 0; kk < n; ++kk) {
      const int k = ord[kk];
      C s(0, 0);
      for (int j = 0; j < n; ++j) s += V[(size_t)r * n + j] * Z[(size_t)j * n + k];
      out[(size_t)r * n + kk] = s;
    }
  for (int kk = 0; kk < n; ++kk) w[kk] = d[ord[kk]];
  V.swap(out);
}

}  // namespace lgw
