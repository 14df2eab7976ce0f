// Small dense FP64 linear algebra for the host-side setup (no LAPACK).
// Row-major storage throughout.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <limits>
#include <thread>
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

// Dot product with four partial sums, so that the loop vectorises without
// reassociation flags.
inline double dot(const double* a, const double* b, size_t n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  size_t k = 0;
  for (; k + 4 <= n; k += 4) {
    s0 += a[k] * b[k];
    s1 += a[k + 1] * b[k + 1];
    s2 += a[k + 2] * b[k + 2];
    s3 += a[k + 3] * b[k + 3];
  }
  for (; k < n; ++k) s0 += a[k] * b[k];
  return (s0 + s1) + (s2 + s3);
}

// y += a x
inline void axpy(double a, const double* x, double* y, size_t n) {
  for (size_t k = 0; k < n; ++k) y[k] += a * x[k];
}

// C[i * ldc + j] (+)= dot(A[i], B[j]) for i < ka, j < kb over n elements:
// the Gram matrix of two sets of row vectors.  Register-blocked 4 x 2 and
// walked in chunks of n so that the rows in use stay in cache.  With
// `lower`, only entries j <= i are guaranteed (for symmetric results; a
// few entries above the diagonal of each 4-row block are also formed).
__attribute__((target_clones("arch=x86-64-v3", "default")))
inline void gram(const double* const* A, int ka, const double* const* B, int kb, size_t n, double* C,
                 size_t ldc, bool accumulate = false, bool lower = false) {
  if (!accumulate)
    for (int i = 0; i < ka; ++i)
      for (int j = 0; j < kb; ++j) C[(size_t)i * ldc + j] = 0.0;
  constexpr size_t kChunk = 512;
  for (size_t t0 = 0; t0 < n; t0 += kChunk) {
    const size_t len = std::min(kChunk, n - t0);
    int i = 0;
    for (; i + 4 <= ka; i += 4) {
      const double *a0 = A[i] + t0, *a1 = A[i + 1] + t0, *a2 = A[i + 2] + t0, *a3 = A[i + 3] + t0;
      const int jend = lower ? std::min(kb, i + 4) : kb;
      int j = 0;
      for (; j + 2 <= jend; j += 2) {
        const double *b0 = B[j] + t0, *b1 = B[j + 1] + t0;
        double s00 = 0, s01 = 0, s10 = 0, s11 = 0, s20 = 0, s21 = 0, s30 = 0, s31 = 0;
        for (size_t t = 0; t < len; ++t) {
          const double x0 = b0[t], x1 = b1[t];
          s00 += a0[t] * x0; s01 += a0[t] * x1;
          s10 += a1[t] * x0; s11 += a1[t] * x1;
          s20 += a2[t] * x0; s21 += a2[t] * x1;
          s30 += a3[t] * x0; s31 += a3[t] * x1;
        }
        C[(size_t)i * ldc + j] += s00; C[(size_t)i * ldc + j + 1] += s01;
        C[(size_t)(i + 1) * ldc + j] += s10; C[(size_t)(i + 1) * ldc + j + 1] += s11;
        C[(size_t)(i + 2) * ldc + j] += s20; C[(size_t)(i + 2) * ldc + j + 1] += s21;
        C[(size_t)(i + 3) * ldc + j] += s30; C[(size_t)(i + 3) * ldc + j + 1] += s31;
      }
      for (; j < jend; ++j) {
        const double* b0 = B[j] + t0;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        for (size_t t = 0; t < len; ++t) {
          s0 += a0[t] * b0[t]; s1 += a1[t] * b0[t]; s2 += a2[t] * b0[t]; s3 += a3[t] * b0[t];
        }
        C[(size_t)i * ldc + j] += s0; C[(size_t)(i + 1) * ldc + j] += s1;
        C[(size_t)(i + 2) * ldc + j] += s2; C[(size_t)(i + 3) * ldc + j] += s3;
      }
    }
    for (; i < ka; ++i)
      for (int j = 0; j < (lower ? std::min(kb, i + 1) : kb); ++j) C[(size_t)i * ldc + j] += dot(A[i] + t0, B[j] + t0, len);
  }
}

// gram() with the rows of A split over host threads when the product is
// large (the setup of models with thousands of states); small products run
// on the calling thread.
inline void gram_mt(const double* const* A, int ka, const double* const* B, int kb, size_t n, double* C,
                    size_t ldc, bool lower = false) {
  const double work = (double)ka * kb * (double)n;
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (work < 2e8 || nt < 2 || ka < 8 * nt) {
    gram(A, ka, B, kb, n, C, ldc, false, lower);
    return;
  }
  std::vector<std::thread> th;
  // rows in chunks of 4 (the register block), balanced by work when lower
  std::vector<int> cut(nt + 1, 0);
  for (int t = 1; t <= nt; ++t) {
    const double f = (double)t / nt;
    int r = lower ? (int)(ka * std::sqrt(f)) : (int)(ka * f);
    cut[t] = std::min(ka, (r + 3) / 4 * 4);
  }
  cut[nt] = ka;
  for (int t = 0; t < nt; ++t) {
    const int r0 = cut[t], r1 = cut[t + 1];
    if (r1 <= r0) continue;
    th.emplace_back([=]() {
      if (lower) {
        // rows r0..r1 need columns up to r1 only
        gram(A + r0, r1 - r0, B, std::min(kb, r1), n, C + (size_t)r0 * ldc, ldc, false, false);
      } else {
        gram(A + r0, r1 - r0, B, kb, n, C + (size_t)r0 * ldc, ldc, false, false);
      }
    });
  }
  for (auto& x : th) x.join();
}

// Y[i] += sum_j C[j * ldc + i] D[j] for i < m, j < k over n elements (a
// linear combination of the rows D applied to every row of Y), four rows
// of D per pass over Y.
__attribute__((target_clones("arch=x86-64-v3", "default")))
inline void add_comb(double* const* Y, int m, const double* const* D, int k, const double* C, size_t ldc,
                     size_t n) {
  constexpr size_t kChunk = 1024;
  for (size_t t0 = 0; t0 < n; t0 += kChunk) {
    const size_t len = std::min(kChunk, n - t0);
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      const double *d0 = D[j] + t0, *d1 = D[j + 1] + t0, *d2 = D[j + 2] + t0, *d3 = D[j + 3] + t0;
      for (int i = 0; i < m; ++i) {
        const double c0 = C[(size_t)j * ldc + i], c1 = C[(size_t)(j + 1) * ldc + i];
        const double c2 = C[(size_t)(j + 2) * ldc + i], c3 = C[(size_t)(j + 3) * ldc + i];
        double* y = Y[i] + t0;
        for (size_t t = 0; t < len; ++t) y[t] += (c0 * d0[t] + c1 * d1[t]) + (c2 * d2[t] + c3 * d3[t]);
      }
    }
    for (; j < k; ++j)
      for (int i = 0; i < m; ++i) axpy(C[(size_t)j * ldc + i], D[j] + t0, Y[i] + t0, len);
  }
}

// Symmetric eigen-decomposition A = Q diag(w) Q^T: Householder reduction to
// tridiagonal form, then implicit symmetric QR steps with Wilkinson shifts
// on the tridiagonal (Golub and Van Loan, Matrix Computations, Sec. 8.3).
// A is destroyed; Q row-major with the eigenvectors as columns; w unsorted.
// Returns false if the QR iteration did not converge.
inline bool sym_eig(int n, double* A, double* Q, double* w) {
  if (n <= 0) return true;
  std::vector<double> d(n), e(n, 0.0), beta(n, 0.0), p(n), wv(n);
  std::vector<double> V((size_t)n * n, 0.0);   // row k: Householder vector on [k+1, n)
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* x = A + (size_t)k * n + k + 1;     // row k right of the diagonal (= column k below it)
    const double nx2 = dot(x, x, m);
    const double tail = nx2 - x[0] * x[0];
    if (tail == 0.0) continue;                 // column already in tridiagonal form
    double* v = V.data() + (size_t)k * n + k + 1;
    const double alpha = x[0] >= 0.0 ? -std::sqrt(nx2) : std::sqrt(nx2);
    for (int i = 0; i < m; ++i) v[i] = x[i];
    v[0] -= alpha;
    const double b = 2.0 / (tail + v[0] * v[0]);
    beta[k] = b;
    // S <- H S H with H = I - b v v^T on the trailing block S = A[k+1:, k+1:]:
    // p = b S v, w = p - (b/2)(p^T v) v, S <- S - v w^T - w v^T
    for (int i = 0; i < m; ++i) p[i] = b * dot(A + (size_t)(k + 1 + i) * n + k + 1, v, m);
    const double K = 0.5 * b * dot(p.data(), v, m);
    for (int i = 0; i < m; ++i) wv[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = A + (size_t)(k + 1 + i) * n + k + 1;
      const double vi = v[i], wi = wv[i];
      for (int j = 0; j < m; ++j) row[j] -= vi * wv[j] + wi * v[j];
    }
    x[0] = alpha;
    for (int i = 1; i < m; ++i) x[i] = 0.0;
    for (int i = 0; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = x[i];
  }
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)i * n + i + 1];
  // Z = H_0 H_1 ... H_{n-3}, accumulated from the right end (each H_k only
  // touches rows and columns k+1..n-1 of the partial product)
  std::vector<double> Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  std::vector<double> u(n);
  for (int k = n - 3; k >= 0; --k) {
    if (beta[k] == 0.0) continue;
    const int m = n - k - 1;
    const double* v = V.data() + (size_t)k * n + k + 1;
    std::fill(u.begin(), u.begin() + m, 0.0);
    for (int i = 0; i < m; ++i) axpy(v[i], Z.data() + (size_t)(k + 1 + i) * n + k + 1, u.data(), m);
    for (int i = 0; i < m; ++i) axpy(-beta[k] * v[i], u.data(), Z.data() + (size_t)(k + 1 + i) * n + k + 1, m);
  }
  // Zt = Z^T: the QR rotations then update two contiguous rows
  std::vector<double> Zt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Zt[(size_t)j * n + i] = Z[(size_t)i * n + j];
  const double eps = std::numeric_limits<double>::epsilon();
  bool ok = true;
  int hi = n - 1, iter = 0;
  while (hi > 0) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 100) {
      ok = false;
      break;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer d[hi]
    const double dl = 0.5 * (d[hi - 1] - d[hi]);
    const double bb = e[hi - 1];
    const double mu = d[hi] - bb * bb / (dl + (dl >= 0.0 ? 1.0 : -1.0) * std::hypot(dl, bb));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // rotation J on (k, k+1), J = [c s; -s c], with s x + c z = 0: the
      // first one acts on the shifted column, the later ones chase the bulge
      const double r = std::hypot(x, z);
      const double c = r > 0.0 ? x / r : 1.0;
      const double s = r > 0.0 ? -z / r : 0.0;
      if (k > lo) e[k - 1] = r;
      const double a = d[k], b2 = d[k + 1], f = e[k];
      d[k] = c * c * a - 2.0 * c * s * f + s * s * b2;
      d[k + 1] = s * s * a + 2.0 * c * s * f + c * c * b2;
      e[k] = c * s * (a - b2) + (c * c - s * s) * f;
      if (k + 1 < hi) {
        x = e[k];
        z = -s * e[k + 1];
        e[k + 1] *= c;
      }
      double* zk = Zt.data() + (size_t)k * n;
      double* zk1 = zk + n;
      for (int i = 0; i < n; ++i) {
        const double a0 = zk[i], a1 = zk1[i];
        zk[i] = c * a0 - s * a1;
        zk1[i] = s * a0 + c * a1;
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = d[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[(size_t)i * n + j] = Zt[(size_t)j * n + i];
  return ok;
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

namespace fdtd {
namespace la {

// add_comb() with the columns split over host threads when the update is
// large; small updates run on the calling thread.
inline void add_comb_mt(double* const* Y, int m, const double* const* D, int k, const double* C, size_t ldc,
                        size_t n) {
  const double work = (double)m * k * (double)n;
  const int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (work < 2e8 || nt < 2 || n < (size_t)nt * 1024) {
    add_comb(Y, m, D, k, C, ldc, n);
    return;
  }
  const size_t chunk = (n + nt - 1) / nt / 1024 * 1024 + 1024;
  std::vector<std::thread> th;
  for (size_t c0 = 0; c0 < n; c0 += chunk) {
    const size_t len = std::min(chunk, n - c0);
    th.emplace_back([=]() {
      std::vector<double*> Yc(m);
      std::vector<const double*> Dc(k);
      for (int i = 0; i < m; ++i) Yc[i] = Y[i] + c0;
      for (int j = 0; j < k; ++j) Dc[j] = D[j] + c0;
      add_comb(Yc.data(), m, Dc.data(), k, C, ldc, len);
    });
  }
  for (auto& x : th) x.join();
}

}  // namespace la
}  // namespace fdtd
