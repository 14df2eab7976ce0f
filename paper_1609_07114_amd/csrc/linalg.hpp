// Small dense FP64 linear algebra for the host-side setup (no LAPACK).
// Row-major storage throughout.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <vector>

namespace fdtd {
namespace la {

// In-place LU with partial pivoting: A = P^T L U.  Returns false if a pivot
// is exactly zero.
inline bool lu_factor(int n, double* A, std::vector<int>& piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      const double v = std::fabs(A[(size_t)r * n + k]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int c = 0; c < n; ++c) std::swap(A[(size_t)k * n + c], A[(size_t)p * n + c]);
    const double inv = 1.0 / A[(size_t)k * n + k];
    for (int r = k + 1; r < n; ++r) {
      double* rowr = A + (size_t)r * n;
      const double f = rowr[k] * inv;
      rowr[k] = f;
      if (f == 0.0) continue;
      const double* rowk = A + (size_t)k * n;
      for (int c = k + 1; c < n; ++c) rowr[c] -= f * rowk[c];
    }
  }
  return true;
}

// Solve A X = B in place for B (n x m) given lu_factor's output.
inline void lu_solve(int n, const double* LU, const std::vector<int>& piv, double* B, int m) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k)
      for (int c = 0; c < m; ++c) std::swap(B[(size_t)k * m + c], B[(size_t)piv[k] * m + c]);
  for (int r = 0; r < n; ++r) {
    double* br = B + (size_t)r * m;
    for (int k = 0; k < r; ++k) {
      const double f = LU[(size_t)r * n + k];
      if (f == 0.0) continue;
      const double* bk = B + (size_t)k * m;
      for (int c = 0; c < m; ++c) br[c] -= f * bk[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double* br = B + (size_t)r * m;
    for (int k = r + 1; k < n; ++k) {
      const double f = LU[(size_t)r * n + k];
      if (f == 0.0) continue;
      const double* bk = B + (size_t)k * m;
      for (int c = 0; c < m; ++c) br[c] -= f * bk[c];
    }
    const double inv = 1.0 / LU[(size_t)r * n + r];
    for (int c = 0; c < m; ++c) br[c] *= inv;
  }
}

// In-place lower Cholesky A = L L^T (lower triangle written).  False if A
// is not numerically positive definite.
inline bool cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    A[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = s / ljj;
    }
  }
  return true;
}

// Cyclic Jacobi eigen-decomposition of a symmetric matrix: A = Q diag(w) Q^T.
// A is destroyed; Q row-major (columns are eigenvectors); w unsorted.
inline void sym_eig(int n, double* A, double* Q, double* w, int max_sweeps = 100) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += A[(size_t)i * n + i] * A[(size_t)i * n + i];
      for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * n + p];
        const double aqq = A[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0);
        const double s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[(size_t)k * n + p];
          const double akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[(size_t)p * n + k];
          const double aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[(size_t)k * n + p];
          const double qkq = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = c * qkp - s * qkq;
          Q[(size_t)k * n + q] = s * qkp + c * qkq;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

// C (m x n) = A (m x k) * B (k x n), all row-major.
inline void gemm(int m, int n, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < m * n; ++i) C[i] = 0.0;
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[(size_t)i * k + l];
      if (a == 0.0) continue;
      const double* b = B + (size_t)l * n;
      double* c = C + (size_t)i * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
}

}  // namespace la
}  // namespace fdtd
