// Host FP64 reduced-model builder (paper Secs. II-III and V-E):
//   fine-region descriptor system on coarse ports -> block Krylov
//   directions -> SPRIM split V = blkdiag(V1, V2) (eq. (9)) -> congruence
//   R~, F~, L~ (eqs. (11)-(12)) -> singular-value clip of eq. (27).
//
// Fine model (eqs. (3)-(8)), restricted to coarse ports (the r fine boundary
// E samples on one coarse interface edge are one unknown, eq. (15)):
//   R = [[De/dt, -K/2], [-K^T/2, Dm/dt]],  F = [[Ds/2, -K/2], [K^T/2, 0]],
//   B = Lc Sc,  Sc = diag(-dx, +dx, +dy, -dy) per port side (S, N, W, E).
// Solves with (p0 R + F) = [[D1, -a K], [b K^T, c I]] (D1 = p0 De/dt + Ds/2,
// a = (1+p0)/2, b = (1-p0)/2, c = p0 Dm/dt) go through the H-block Schur
// complement S = c I + a b K^T D1^{-1} K, which is symmetric positive
// definite for 0 < p0 < 1; S is banded in the natural cell order and is
// factored once by a banded Cholesky.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdtd_rom.h"
#include "common.hpp"
#include "linalg.hpp"

namespace {

const double kC0 = FDTD_C0;
const double kMu0 = FDTD_MU0;
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

struct Csr {
  int rows = 0, cols = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

Csr transpose(const Csr& A) {
  Csr T;
  T.rows = A.cols;
  T.cols = A.rows;
  T.ptr.assign(T.rows + 1, 0);
  for (int c : A.col) T.ptr[c + 1]++;
  for (int r = 0; r < T.rows; ++r) T.ptr[r + 1] += T.ptr[r];
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  std::vector<int> fill(T.ptr.begin(), T.ptr.end() - 1);
  for (int r = 0; r < A.rows; ++r)
    for (int k = A.ptr[r]; k < A.ptr[r + 1]; ++k) {
      const int d = fill[A.col[k]]++;
      T.col[d] = r;
      T.val[d] = A.val[k];
    }
  return T;
}

// out (A.rows) = A x (A.cols), one column
void spmv(const Csr& A, const double* x, double* out) {
  for (int r = 0; r < A.rows; ++r) {
    double s = 0;
    for (int k = A.ptr[r]; k < A.ptr[r + 1]; ++k) s += A.val[k] * x[A.col[k]];
    out[r] = s;
  }
}

struct FineModel {
  int Nx, Ny, ni, nj, r, np;
  int nEx, nEy, nE, nH, n;
  double dx, dy, dxh, dyh, dt;
  std::vector<double> De, Ds, Sc;  // E diagonals, port scale
  // per E coordinate the fine cells whose half cells make it up:
  // De = sum w eps0 eps_r(cell), Ds = sum w sigma(cell)
  std::vector<std::vector<std::pair<int, double>>> ecells;
  double Dm;
  Csr K, KT;                       // E x H and its transpose
  std::vector<int> port_row;       // E index of each port
};

// Restricted fine model.  E order: interior Ex (j = 1..Ny-1, i), interior Ey
// (j, i = 1..Nx-1), ports S, N, W, E; H order: j * Nx + i.  Samples on PEC
// fine cells (pec != nullptr: the cell's Hz and its four edges) are pinned to
// zero and left out of the state; a coarse port whose r fine edges are all
// pinned has no coordinate (port_row = -1).  Returns false, with a message,
// when a port has only some of its fine edges pinned.
bool assemble(FineModel& m, int ni, int nj, int r, double dx, double dy, double dt, const double* er,
              const double* sg, const uint8_t* pec, std::string& err) {
  m.ni = ni;
  m.nj = nj;
  m.r = r;
  m.Nx = r * ni;
  m.Ny = r * nj;
  m.dx = dx;
  m.dy = dy;
  m.dt = dt;
  m.dxh = dx / r;
  m.dyh = dy / r;
  const int Nx = m.Nx, Ny = m.Ny;
  m.np = 2 * (ni + nj);
  auto metal = [&](int i, int j) { return pec && i >= 0 && i < Nx && j >= 0 && j < Ny && pec[(size_t)j * Nx + i]; };
  // pinned edges: a side of a PEC cell
  auto pin_x = [&](int i, int j) { return metal(i, j - 1) || metal(i, j); };   // Ex(i, j)
  auto pin_y = [&](int i, int j) { return metal(i - 1, j) || metal(i, j); };   // Ey(i, j)
  // H coordinates
  std::vector<int> hid((size_t)Nx * Ny, -1);
  m.nH = 0;
  for (int j = 0; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i)
      if (!metal(i, j)) hid[(size_t)j * Nx + i] = m.nH++;
  // port liveness (all r fine edges free, or all pinned)
  std::vector<char> live(m.np, 1);
  for (int c = 0; c < m.np; ++c) {
    int npin = 0;
    for (int k = 0; k < r; ++k) {
      bool p;
      if (c < ni) p = pin_x(c * r + k, 0);
      else if (c < 2 * ni) p = pin_x((c - ni) * r + k, Ny);
      else if (c < 2 * ni + nj) p = pin_y(0, (c - 2 * ni) * r + k);
      else p = pin_y(Nx, (c - 2 * ni - nj) * r + k);
      npin += p ? 1 : 0;
    }
    if (npin != 0 && npin != r) {
      err = "coarse port " + std::to_string(c) + ": only some of its fine edges lie on PEC cells";
      return false;
    }
    live[c] = npin == 0;
  }
  m.De.clear();
  m.Ds.clear();
  m.Dm = kMu0 * m.dxh * m.dyh;
  const double A = m.dxh * m.dyh;
  auto E = [&](int i, int j) { return er[(size_t)j * Nx + i]; };
  auto S = [&](int i, int j) { return sg[(size_t)j * Nx + i]; };
  auto H = [&](int i, int j) { return hid[(size_t)j * Nx + i]; };
  std::vector<std::vector<std::pair<int, double>>> rows;
  m.ecells.clear();
  auto cell = [&](int i, int j) { return j * Nx + i; };
  auto add_e = [&](double de, double ds, std::vector<std::pair<int, double>> k,
                   std::vector<std::pair<int, double>> cells) {
    m.De.push_back(de);
    m.Ds.push_back(ds);
    rows.push_back(std::move(k));
    m.ecells.push_back(std::move(cells));
  };
  for (int j = 1; j < Ny; ++j)
    for (int i = 0; i < Nx; ++i)
      if (!pin_x(i, j))
        add_e(A * kEps0 * 0.5 * (E(i, j - 1) + E(i, j)), A * 0.5 * (S(i, j - 1) + S(i, j)),
              {{H(i, j), +m.dxh}, {H(i, j - 1), -m.dxh}}, {{cell(i, j - 1), 0.5 * A}, {cell(i, j), 0.5 * A}});
  m.nEx = (int)rows.size();
  for (int j = 0; j < Ny; ++j)
    for (int i = 1; i < Nx; ++i)
      if (!pin_y(i, j))
        add_e(A * kEps0 * 0.5 * (E(i - 1, j) + E(i, j)), A * 0.5 * (S(i - 1, j) + S(i, j)),
              {{H(i, j), -m.dyh}, {H(i - 1, j), +m.dyh}}, {{cell(i - 1, j), 0.5 * A}, {cell(i, j), 0.5 * A}});
  m.nEy = (int)rows.size() - m.nEx;
  m.Sc.assign(m.np, 0.0);
  m.port_row.assign(m.np, -1);
  for (int c = 0; c < ni; ++c) {
    m.Sc[c] = -dx;
    m.Sc[ni + c] = +dx;
  }
  for (int c = 0; c < nj; ++c) {
    m.Sc[2 * ni + c] = +dy;
    m.Sc[2 * ni + nj + c] = -dy;
  }
  for (int c = 0; c < m.np; ++c) {
    if (!live[c]) continue;
    // boundary half cells of eq. (4), summed over the r fine edges
    double de = 0, ds = 0;
    std::vector<std::pair<int, double>> k, cells;
    for (int t = 0; t < r; ++t) {
      if (c < ni) {
        const int i = c * r + t;
        de += m.dxh * (m.dyh / 2) * kEps0 * E(i, 0);
        ds += m.dxh * (m.dyh / 2) * S(i, 0);
        k.push_back({H(i, 0), +m.dxh});
        cells.push_back({cell(i, 0), m.dxh * (m.dyh / 2)});
      } else if (c < 2 * ni) {
        const int i = (c - ni) * r + t;
        de += m.dxh * (m.dyh / 2) * kEps0 * E(i, Ny - 1);
        ds += m.dxh * (m.dyh / 2) * S(i, Ny - 1);
        k.push_back({H(i, Ny - 1), -m.dxh});
        cells.push_back({cell(i, Ny - 1), m.dxh * (m.dyh / 2)});
      } else if (c < 2 * ni + nj) {
        const int j = (c - 2 * ni) * r + t;
        de += m.dyh * (m.dxh / 2) * kEps0 * E(0, j);
        ds += m.dyh * (m.dxh / 2) * S(0, j);
        k.push_back({H(0, j), -m.dyh});
        cells.push_back({cell(0, j), m.dyh * (m.dxh / 2)});
      } else {
        const int j = (c - 2 * ni - nj) * r + t;
        de += m.dyh * (m.dxh / 2) * kEps0 * E(Nx - 1, j);
        ds += m.dyh * (m.dxh / 2) * S(Nx - 1, j);
        k.push_back({H(Nx - 1, j), +m.dyh});
        cells.push_back({cell(Nx - 1, j), m.dyh * (m.dxh / 2)});
      }
    }
    m.port_row[c] = (int)rows.size();
    add_e(de, ds, std::move(k), std::move(cells));
  }
  m.nE = (int)rows.size();
  m.n = m.nE + m.nH;
  m.K.rows = m.nE;
  m.K.cols = m.nH;
  m.K.ptr.assign(m.nE + 1, 0);
  for (int e = 0; e < m.nE; ++e) {
    for (auto& pr : rows[e]) {
      // every Hz next to a free edge is free (a PEC cell pins all its edges)
      m.K.col.push_back(pr.first);
      m.K.val.push_back(pr.second);
    }
    m.K.ptr[e + 1] = (int)m.K.col.size();
  }
  m.KT = transpose(m.K);
  return true;
}

// Banded Cholesky of an SPD matrix with half-bandwidth bw; L(i, i-d) at
// L[i*(bw+1) + d].
struct Banded {
  int n = 0, bw = 0;
  std::vector<double> L;
  double& at(int i, int d) { return L[(size_t)i * (bw + 1) + d]; }
  double get(int i, int j) const { return L[(size_t)i * (bw + 1) + (i - j)]; }
};

bool band_cholesky(Banded& B) {
  const int n = B.n, bw = B.bw, w = bw + 1;
  double* L = B.L.data();
  for (int i = 0; i < n; ++i) {
    const int j0 = std::max(0, i - bw);
    for (int j = j0; j <= i; ++j) {
      double s = L[(size_t)i * w + (i - j)];
      const int k0 = std::max(j0, j - bw);
      const double* li = L + (size_t)i * w;
      const double* lj = L + (size_t)j * w;
      for (int k = k0; k < j; ++k) s -= li[i - k] * lj[j - k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[(size_t)i * w] = std::sqrt(s);
      } else {
        L[(size_t)i * w + (i - j)] = s / lj[0];
      }
    }
  }
  return true;
}

void band_solve(const Banded& B, double* x) {
  const int n = B.n, bw = B.bw, w = bw + 1;
  const double* L = B.L.data();
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    const double* li = L + (size_t)i * w;
    const int k0 = std::max(0, i - bw);
    for (int k = k0; k < i; ++k) s -= li[i - k] * x[k];
    x[i] = s / li[0];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    const int k1 = std::min(n - 1, i + bw);
    for (int k = i + 1; k <= k1; ++k) s -= L[(size_t)k * w + (k - i)] * x[k];
    x[i] = s / L[(size_t)i * w];
  }
}

struct Solver {
  const FineModel* m;
  double p0, a, b, c;
  std::vector<double> D1;
  Banded S;
  std::vector<double> t, u, v;

  bool init(const FineModel& fm, double p0_) {
    m = &fm;
    p0 = p0_;
    a = 0.5 * (1.0 + p0);
    b = 0.5 * (1.0 - p0);
    c = p0 * fm.Dm / fm.dt;
    D1.resize(fm.nE);
    for (int e = 0; e < fm.nE; ++e) D1[e] = p0 * fm.De[e] / fm.dt + 0.5 * fm.Ds[e];
    // bandwidth of K^T D1^{-1} K
    int bw = 0;
    for (int e = 0; e < fm.nE; ++e)
      for (int k = fm.K.ptr[e]; k < fm.K.ptr[e + 1]; ++k)
        for (int l = fm.K.ptr[e]; l < fm.K.ptr[e + 1]; ++l)
          bw = std::max(bw, std::abs(fm.K.col[k] - fm.K.col[l]));
    S.n = fm.nH;
    S.bw = bw;
    S.L.assign((size_t)fm.nH * (bw + 1), 0.0);
    for (int h = 0; h < fm.nH; ++h) S.at(h, 0) = c;
    for (int e = 0; e < fm.nE; ++e) {
      const double wgt = a * b / D1[e];
      for (int k = fm.K.ptr[e]; k < fm.K.ptr[e + 1]; ++k)
        for (int l = fm.K.ptr[e]; l < fm.K.ptr[e + 1]; ++l) {
          const int i = fm.K.col[k], j = fm.K.col[l];
          if (j > i) continue;
          S.at(i, i - j) += wgt * fm.K.val[k] * fm.K.val[l];
        }
    }
    t.resize(fm.nE);
    u.resize(fm.nH);
    v.resize(fm.nE);
    return band_cholesky(S);
  }

  // x = (p0 R + F)^{-1} rhs, one column of length n (E part then H part)
  void solve(const double* rhs, double* x) {
    const FineModel& fm = *m;
    for (int e = 0; e < fm.nE; ++e) t[e] = rhs[e] / D1[e];
    spmv(fm.KT, t.data(), u.data());
    double* xh = x + fm.nE;
    for (int h = 0; h < fm.nH; ++h) xh[h] = rhs[fm.nE + h] - b * u[h];
    band_solve(S, xh);
    spmv(fm.K, xh, v.data());
    for (int e = 0; e < fm.nE; ++e) x[e] = t[e] + a * v[e] / D1[e];
  }

  // y = R x, one column
  void apply_R(const double* x, double* y) {
    const FineModel& fm = *m;
    spmv(fm.K, x + fm.nE, v.data());
    spmv(fm.KT, x, u.data());
    for (int e = 0; e < fm.nE; ++e) y[e] = fm.De[e] / fm.dt * x[e] - 0.5 * v[e];
    for (int h = 0; h < fm.nH; ++h) y[fm.nE + h] = -0.5 * u[h] + fm.Dm / fm.dt * x[fm.nE + h];
  }
};

using Cols = std::vector<std::vector<double>>;  // column vectors

// Krylov directions, ordered as described in rom builder docs.
bool krylov_dirs(Solver& sol, const FineModel& fm, int ncols, Cols& dirs, std::string& err) {
  const int n = fm.n;
  std::vector<double> mass(n);
  for (int e = 0; e < fm.nE; ++e) mass[e] = fm.De[e] / fm.dt;
  for (int h = 0; h < fm.nH; ++h) mass[fm.nE + h] = fm.Dm / fm.dt;
  // X0 = (p0 R + F)^{-1} B, B = Lc Sc
  Cols X(fm.np, std::vector<double>(n, 0.0));
  std::vector<double> rhs(n);
  for (int p = 0; p < fm.np; ++p) {
    if (fm.port_row[p] < 0) continue;  // port pinned by PEC: no input (zero column, deflated)
    std::fill(rhs.begin(), rhs.end(), 0.0);
    rhs[fm.port_row[p]] = fm.Sc[p];
    sol.solve(rhs.data(), X[p].data());
  }
  double ref = -1;
  const double tol = 1e-12;
  Cols MX;
  std::vector<double> C;
  while ((int)dirs.size() < ncols) {
    const int m = (int)X.size();
    std::vector<double*> Xp(m);
    std::vector<const double*> MXp(m);
    MX.assign(m, std::vector<double>(n));
    for (int i = 0; i < m; ++i) {
      Xp[i] = X[i].data();
      MXp[i] = MX[i].data();
    }
    auto weigh = [&]() {
      for (int i = 0; i < m; ++i)
        for (int k = 0; k < n; ++k) MX[i][k] = mass[k] * X[i][k];
    };
    // two passes of mass-orthogonalisation of the block against all
    // earlier directions: X -= D (D^T M X)
    if (!dirs.empty()) {
      const int kd = (int)dirs.size();
      std::vector<const double*> Dp(kd);
      for (int j = 0; j < kd; ++j) Dp[j] = dirs[j].data();
      C.resize((size_t)kd * m);
      for (int pass = 0; pass < 2; ++pass) {
        weigh();
        fdtd::la::gram_mt(Dp.data(), kd, MXp.data(), m, n, C.data(), m);
        for (double& c : C) c = -c;
        fdtd::la::add_comb_mt(Xp.data(), m, Dp.data(), kd, C.data(), m, n);
      }
    }
    std::vector<double> G((size_t)m * m), Q((size_t)m * m), w(m);
    weigh();
    std::vector<const double*> Xc(Xp.begin(), Xp.end());
    fdtd::la::gram(Xc.data(), m, MXp.data(), m, n, G.data(), m, false, true);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < i; ++j) G[(size_t)j * m + i] = G[(size_t)i * m + j];
    if (!fdtd::la::sym_eig(m, G.data(), Q.data(), w.data())) {
      err = "eigen-decomposition of a Krylov block did not converge";
      return false;
    }
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });
    if (ref < 0) ref = w[order[0]];
    // new directions: eigenvectors of the block's mass Gram matrix in
    // decreasing order, W_o = X z_o / sqrt(w_o)
    int nw = 0;
    while (nw < m && w[order[nw]] > tol * tol * ref) ++nw;
    Cols W(nw, std::vector<double>(n, 0.0));
    if (nw > 0) {
      std::vector<double*> Wp(nw);
      for (int o = 0; o < nw; ++o) Wp[o] = W[o].data();
      std::vector<double> Z((size_t)m * nw);
      for (int j = 0; j < m; ++j)
        for (int o = 0; o < nw; ++o) Z[(size_t)j * nw + o] = Q[(size_t)j * m + order[o]] / std::sqrt(w[order[o]]);
      fdtd::la::add_comb_mt(Wp.data(), nw, Xc.data(), m, Z.data(), nw, n);
    }
    if (W.empty()) break;
    if (dirs.size() + W.size() >= (size_t)ncols) {
      for (auto& v : W) dirs.push_back(std::move(v));
      break;
    }
    Cols Xn(W.size(), std::vector<double>(n));
    std::vector<double> Rw(n);
    for (size_t c = 0; c < W.size(); ++c) {
      sol.apply_R(W[c].data(), Rw.data());
      sol.solve(Rw.data(), Xn[c].data());
    }
    for (auto& v : W) dirs.push_back(std::move(v));
    X.swap(Xn);
  }
  return true;
}

// Gram-Schmidt in order over rows [r0, r0+len) of the directions: each
// direction, orthogonalised (two passes) against the ones already kept, is
// kept if its residual stays above 1e-10 of its norm, until q are kept.
// Worked in blocks of 32 directions: two block passes against the vectors
// kept before the block, then in order within the block.
Cols gs_part(const Cols& dirs, int r0, int len, int q) {
  Cols out;
  constexpr size_t kB = 32;
  std::vector<double> C;
  for (size_t next = 0; next < dirs.size() && (int)out.size() < q; next += kB) {
    const int b = (int)std::min(kB, dirs.size() - next);
    Cols blk(b);
    std::vector<double> nv(b);
    std::vector<double*> Bp(b);
    for (int i = 0; i < b; ++i) {
      blk[i].assign(dirs[next + i].begin() + r0, dirs[next + i].begin() + r0 + len);
      nv[i] = std::sqrt(fdtd::la::dot(blk[i].data(), blk[i].data(), len));
      Bp[i] = blk[i].data();
    }
    if (!out.empty()) {
      const int k = (int)out.size();
      std::vector<const double*> U(k);
      for (int j = 0; j < k; ++j) U[j] = out[j].data();
      C.resize((size_t)k * b);
      std::vector<const double*> Bc(Bp.begin(), Bp.end());
      for (int pass = 0; pass < 2; ++pass) {
        fdtd::la::gram_mt(U.data(), k, Bc.data(), b, len, C.data(), b);
        for (double& c : C) c = -c;
        fdtd::la::add_comb_mt(Bp.data(), b, U.data(), k, C.data(), b, len);
      }
    }
    const size_t first = out.size();
    for (int i = 0; i < b && (int)out.size() < q; ++i) {
      if (nv[i] == 0.0) continue;
      double* v = blk[i].data();
      for (int pass = 0; pass < 2; ++pass)
        for (size_t u = first; u < out.size(); ++u)
          fdtd::la::axpy(-fdtd::la::dot(out[u].data(), v, len), out[u].data(), v, len);
      const double nr = std::sqrt(fdtd::la::dot(v, v, len));
      if (nr <= 1e-10 * nv[i]) continue;
      for (int t = 0; t < len; ++t) v[t] /= nr;
      out.push_back(std::move(blk[i]));
    }
  }
  return out;
}

// What the gradient through the builder needs of a build.
struct BuildState {
  FineModel fm;
  Cols V1;                 // E basis (empty: identity)
  std::vector<double> K0;  // K~ before the clip, q1 x q2
  int q1 = 0, q2 = 0;
  bool clipped = false;
  double lim = 0;
};

int build_impl(const fdtd_rom_build_params* prm, double* Rt, double* Ft, double* Lt, fdtd_rom_build_info* info,
               BuildState* bs);

}  // namespace

using fdtd::fail;

namespace {

int build_impl(const fdtd_rom_build_params* prm, double* Rt, double* Ft, double* Lt, fdtd_rom_build_info* info,
               BuildState* bs) {
  if (!prm) return fail(FDTD_EINVAL, "null argument");
  const bool query = !Rt && !Ft && !Lt;
  if (query ? !info : (!Rt || !Ft || !Lt)) return fail(FDTD_EINVAL, "null argument");
  const fdtd_rom_build_params& P = *prm;
  if (P.ni < 1 || P.nj < 1 || P.r < 1) return fail(FDTD_EINVAL, "bad region size");
  if (!(P.dx > 0) || !(P.dy > 0) || !(P.dt > 0)) return fail(FDTD_EINVAL, "dx, dy, dt must be positive");
  if (!P.eps_r || !P.sigma) return fail(FDTD_EINVAL, "fine material maps required");
  if (P.basis != 0 && P.basis != 1) return fail(FDTD_EINVAL, "basis must be 0 (SPRIM) or 1 (identity)");
  const bool ident = P.basis == 1;
  if (!ident && !query && P.q < 2) return fail(FDTD_EINVAL, "order q must be >= 2");
  const double p0 = 3.14159265358979323846 * P.f_max * P.dt;
  if (!ident && !(p0 > 0.0 && p0 < 1.0))
    return fail(FDTD_EINVAL, "expansion point p0 = pi f_max dt = %g outside (0, 1)", p0);
  const double theta = P.theta > 0 ? P.theta : 0.99;
  const size_t nf = (size_t)P.r * P.ni * P.r * P.nj;
  for (size_t k = 0; k < nf; ++k)
    if (!(P.eps_r[k] > 0) || !(P.sigma[k] >= 0)) return fail(FDTD_EINVAL, "fine material must have eps_r > 0, sigma >= 0");
  try {
    FineModel fm;
    {
      std::string err;
      if (!assemble(fm, P.ni, P.nj, P.r, P.dx, P.dy, P.dt, P.eps_r, P.sigma, P.pec, err))
        return fail(FDTD_EINVAL, "%s", err.c_str());
    }
    const int q1 = ident ? fm.nE : (P.q + 1) / 2, q2 = ident ? fm.nH : P.q / 2;
    if (query) {
      info->q1 = q1;
      info->q2 = q2;
      info->p0 = p0;
      info->smax_before = info->smax_after = 0.0;
      info->clipped = 0;
      info->n_fine_states = fm.n;
      return FDTD_OK;
    }
    if (ident && P.q != fm.n)
      return fail(FDTD_EINVAL, "identity basis: q must equal the restricted state count %d (got %d)", fm.n, P.q);
    if (q1 > fm.nE || q2 > fm.nH) return fail(FDTD_EINVAL, "order q=%d exceeds the fine model", P.q);
    const int q = q1 + q2, np = fm.np;
    double* R = Rt;  // written in place: R~ and F~ of eqs. (11)-(12), q x q row-major
    double* F = Ft;
    std::fill(R, R + (size_t)q * q, 0.0);
    std::fill(F, F + (size_t)q * q, 0.0);
    std::vector<double> Kt((size_t)q1 * q2, 0.0);  // K~ = V1^T K V2
    Cols V1;
    if (ident) {
      // V = I: R~ = R, F~ = F, L~ = Lc of the restricted fine model
      for (int e = 0; e < q1; ++e) {
        R[(size_t)e * q + e] = fm.De[e] / P.dt;
        F[(size_t)e * q + e] = 0.5 * fm.Ds[e];
        for (int k = fm.K.ptr[e]; k < fm.K.ptr[e + 1]; ++k) Kt[(size_t)e * q2 + fm.K.col[k]] = fm.K.val[k];
      }
      for (int h = 0; h < q2; ++h) R[(size_t)(q1 + h) * q + q1 + h] = fm.Dm / P.dt;
    } else {
      Solver sol;
      if (!sol.init(fm, p0)) return fail(FDTD_EINVAL, "Schur complement not positive definite");
      Cols dirs;
      std::string err;
      const int need = std::max(q1, q2);
      if (!krylov_dirs(sol, fm, need + 8, dirs, err)) return fail(FDTD_EINVAL, "%s", err.c_str());
      V1 = gs_part(dirs, 0, fm.nE, q1);
      Cols V2 = gs_part(dirs, fm.nE, fm.nH, q2);
      if ((int)V1.size() < q1 || (int)V2.size() < q2)
        return fail(FDTD_EINVAL, "Krylov space too small for q=%d (got %zu E, %zu H)", P.q, V1.size(), V2.size());
      // congruence (eqs. (11)-(12))
      {
        Cols VD(q1, std::vector<double>(fm.nE)), VS(q1, std::vector<double>(fm.nE));
        std::vector<const double*> V1p(q1), VDp(q1), VSp(q1);
        for (int a = 0; a < q1; ++a) {
          for (int e = 0; e < fm.nE; ++e) {
            VD[a][e] = V1[a][e] * fm.De[e];
            VS[a][e] = V1[a][e] * fm.Ds[e];
          }
          V1p[a] = V1[a].data();
          VDp[a] = VD[a].data();
          VSp[a] = VS[a].data();
        }
        std::vector<double> GR((size_t)q1 * q1), GF((size_t)q1 * q1);
        fdtd::la::gram_mt(VDp.data(), q1, V1p.data(), q1, fm.nE, GR.data(), q1, true);
        fdtd::la::gram_mt(VSp.data(), q1, V1p.data(), q1, fm.nE, GF.data(), q1, true);
        for (int a = 0; a < q1; ++a)
          for (int b2 = 0; b2 <= a; ++b2) {
            R[(size_t)a * q + b2] = R[(size_t)b2 * q + a] = GR[(size_t)a * q1 + b2] / P.dt;
            F[(size_t)a * q + b2] = F[(size_t)b2 * q + a] = 0.5 * GF[(size_t)a * q1 + b2];
          }
      }
      {
        Cols KV(q2, std::vector<double>(fm.nE));
        std::vector<const double*> KVp(q2), V1p(q1), V2p(q2);
        for (int c = 0; c < q2; ++c) {
          spmv(fm.K, V2[c].data(), KV[c].data());
          KVp[c] = KV[c].data();
          V2p[c] = V2[c].data();
        }
        for (int a = 0; a < q1; ++a) V1p[a] = V1[a].data();
        fdtd::la::gram_mt(V1p.data(), q1, KVp.data(), q2, fm.nE, Kt.data(), q2);
        std::vector<double> GH((size_t)q2 * q2);
        fdtd::la::gram_mt(V2p.data(), q2, V2p.data(), q2, fm.nH, GH.data(), q2, true);
        for (int a = 0; a < q2; ++a)
          for (int b2 = 0; b2 <= a; ++b2)
            R[(size_t)(q1 + a) * q + q1 + b2] = R[(size_t)(q1 + b2) * q + q1 + a] = fm.Dm / P.dt * GH[(size_t)a * q2 + b2];
      }
    }
    if (bs) bs->K0 = Kt;
    // eq. (27): singular values s_k of R11^{-1/2} K~ R22^{-1/2} against 2/dt.
    // With Cholesky factors R11 = L1 L1^T, R22 = L2 L2^T the matrix
    // M = L1^{-1} K~ L2^{-T} is orthogonally equivalent to it (R^{1/2} =
    // L Omega with Omega orthogonal), and lowering singular values commutes
    // with orthogonal factors, so K~' = L1 clip(M) L2^T is the same update.
    // Diagonal R11 or R22 (the identity basis) make the factors scalings.
    auto block_diag = [&](int o, int n) {
      for (int a = 0; a < n; ++a)
        for (int b2 = 0; b2 < n; ++b2)
          if (a != b2 && R[(size_t)(o + a) * q + o + b2] != 0.0) return false;
      return true;
    };
    const bool d1 = block_diag(0, q1), d2 = block_diag(q1, q2);
    std::vector<double> L1, L2;  // dense lower factors, or the diagonal of the factor
    auto factor = [&](int o, int n, bool diag, std::vector<double>& L) {
      if (diag) {
        L.resize(n);
        for (int a = 0; a < n; ++a) {
          const double v = P.dt * R[(size_t)(o + a) * q + o + a];
          if (!(v > 0.0)) return false;
          L[a] = std::sqrt(v);
        }
        return true;
      }
      L.assign((size_t)n * n, 0.0);
      for (int a = 0; a < n; ++a)
        for (int b2 = 0; b2 < n; ++b2) L[(size_t)a * n + b2] = P.dt * R[(size_t)(o + a) * q + o + b2];
      return fdtd::la::cholesky(n, L.data());
    };
    if (!factor(0, q1, d1, L1) || !factor(q1, q2, d2, L2))
      return fail(FDTD_EINVAL, "reduced R~ not positive definite (basis lost rank)");
    // M = L1^{-1} K~ L2^{-T}: rows by forward substitution with L1, then each
    // row m solves L2 m^T = x^T
    std::vector<double> M(Kt);
    for (int a = 0; a < q1; ++a) {
      double* xa = M.data() + (size_t)a * q2;
      if (!d1)
        for (int b2 = 0; b2 < a; ++b2) fdtd::la::axpy(-L1[(size_t)a * q1 + b2], M.data() + (size_t)b2 * q2, xa, q2);
      const double inv = 1.0 / (d1 ? L1[a] : L1[(size_t)a * q1 + a]);
      for (int c = 0; c < q2; ++c) xa[c] *= inv;
    }
    for (int a = 0; a < q1; ++a) {
      double* ma = M.data() + (size_t)a * q2;
      if (d2)
        for (int c = 0; c < q2; ++c) ma[c] /= L2[c];
      else
        for (int c = 0; c < q2; ++c) ma[c] = (ma[c] - fdtd::la::dot(L2.data() + (size_t)c * q2, ma, c)) / L2[(size_t)c * q2 + c];
    }
    // M^T M by rank-one row updates (rows of a sparse M cost their nonzeros)
    std::vector<double> MtM((size_t)q2 * q2, 0.0), Wv((size_t)q2 * q2), s2(q2);
    for (int a = 0; a < q1; ++a) {
      const double* ma = M.data() + (size_t)a * q2;
      for (int i = 0; i < q2; ++i)
        if (ma[i] != 0.0) fdtd::la::axpy(ma[i], ma, MtM.data() + (size_t)i * q2, q2);
    }
    if (!fdtd::la::sym_eig(q2, MtM.data(), Wv.data(), s2.data()))
      return fail(FDTD_EINVAL, "eigen-decomposition for the CFL clip did not converge");
    double smax = 0;
    for (int k = 0; k < q2; ++k) smax = std::max(smax, std::sqrt(std::max(0.0, s2[k])));
    const double lim = theta * 2.0 / P.dt;
    double smax_after = smax;
    int clipped = 0;
    if (P.clip && smax > lim) {
      clipped = 1;
      smax_after = 0;
      // lowering s_k to lim along the right singular vector w_k is
      // M <- M (I - sum_k d_k w_k w_k^T), d_k = (s_k - lim) / s_k (the w_k
      // are orthonormal, so the rank-one changes do not interact)
      std::vector<int> cl;
      for (int k = 0; k < q2; ++k) {
        const double sk = std::sqrt(std::max(0.0, s2[k]));
        if (sk > lim) cl.push_back(k);
        smax_after = std::max(smax_after, std::min(sk, lim));
      }
      const int nc = (int)cl.size();
      Cols Wc(q2, std::vector<double>(nc));
      std::vector<const double*> Wp(q2);
      for (int i = 0; i < q2; ++i) {
        for (int c = 0; c < nc; ++c) {
          const double sk = std::sqrt(s2[cl[c]]);
          Wc[i][c] = Wv[(size_t)i * q2 + cl[c]] * std::sqrt((sk - lim) / sk);
        }
        Wp[i] = Wc[i].data();
      }
      std::vector<double> Pm((size_t)q2 * q2);
      fdtd::la::gram_mt(Wp.data(), q2, Wp.data(), q2, nc, Pm.data(), q2);
      for (size_t k = 0; k < Pm.size(); ++k) Pm[k] = -Pm[k];
      for (int i = 0; i < q2; ++i) Pm[(size_t)i * q2 + i] += 1.0;
      // M' = M P row by row over each row's nonzeros; then K~ = L1 M' L2^T
      std::vector<double> Mc((size_t)q1 * q2, 0.0);
      for (int a = 0; a < q1; ++a) {
        const double* ma = M.data() + (size_t)a * q2;
        double* out = Mc.data() + (size_t)a * q2;
        for (int i = 0; i < q2; ++i)
          if (ma[i] != 0.0) fdtd::la::axpy(ma[i], Pm.data() + (size_t)i * q2, out, q2);
      }
      std::vector<double> T;
      if (d1) {
        for (int a = 0; a < q1; ++a)
          for (int c = 0; c < q2; ++c) Mc[(size_t)a * q2 + c] *= L1[a];
      } else {
        T.assign((size_t)q1 * q2, 0.0);
        for (int a = 0; a < q1; ++a)
          for (int b2 = 0; b2 <= a; ++b2)
            fdtd::la::axpy(L1[(size_t)a * q1 + b2], Mc.data() + (size_t)b2 * q2, T.data() + (size_t)a * q2, q2);
        Mc.swap(T);
      }
      for (int a = 0; a < q1; ++a)
        for (int c = 0; c < q2; ++c)
          Kt[(size_t)a * q2 + c] = d2 ? Mc[(size_t)a * q2 + c] * L2[c]
                                      : fdtd::la::dot(Mc.data() + (size_t)a * q2, L2.data() + (size_t)c * q2, c + 1);
    }
    for (int a = 0; a < q1; ++a)
      for (int c = 0; c < q2; ++c) {
        const double k = Kt[(size_t)a * q2 + c];
        R[(size_t)a * q + q1 + c] = -0.5 * k;
        R[(size_t)(q1 + c) * q + a] = -0.5 * k;
        F[(size_t)a * q + q1 + c] = -0.5 * k;
        F[(size_t)(q1 + c) * q + a] = +0.5 * k;
      }
    for (int a = 0; a < q; ++a)
      for (int p = 0; p < np; ++p)
        Lt[(size_t)a * np + p] = (a >= q1 || fm.port_row[p] < 0) ? 0.0
                                 : ident ? (a == fm.port_row[p] ? 1.0 : 0.0) : V1[a][fm.port_row[p]];
    if (info) {
      info->q1 = q1;
      info->q2 = q2;
      info->p0 = p0;
      info->smax_before = smax;
      info->smax_after = smax_after;
      info->clipped = clipped;
      info->n_fine_states = fm.n;
    }
    if (bs) {
      bs->q1 = q1;
      bs->q2 = q2;
      bs->clipped = clipped != 0;
      bs->lim = lim;
      bs->V1 = std::move(V1);
      bs->fm = std::move(fm);
    }
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

}  // namespace

extern "C" int fdtd_rom_build(const fdtd_rom_build_params* prm, double* Rt, double* Ft, double* Lt,
                              fdtd_rom_build_info* info) {
  return build_impl(prm, Rt, Ft, Lt, info, nullptr);
}

namespace {

using Mat = std::vector<double>;  // dense, row-major

Mat mul(const Mat& A, const Mat& B, int m, int k, int n) {  // (m x k)(k x n)
  Mat C((size_t)m * n);
  fdtd::la::gemm(m, n, k, A.data(), B.data(), C.data());
  return C;
}

Mat tr(const Mat& A, int m, int n) {  // (m x n)^T
  Mat T((size_t)n * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) T[(size_t)j * m + i] = A[(size_t)i * n + j];
  return T;
}

// Symmetric eigen-decomposition S = Z diag(w) Z^T (Z columns).  Diagonal
// matrices skip the iteration.
bool eig(int n, const Mat& S, Mat& Z, std::vector<double>& w) {
  bool diag = true;
  for (int i = 0; i < n && diag; ++i)
    for (int j = 0; j < n && diag; ++j) diag = i == j || S[(size_t)i * n + j] == 0.0;
  Z.assign((size_t)n * n, 0.0);
  w.resize(n);
  if (diag) {
    for (int i = 0; i < n; ++i) {
      Z[(size_t)i * n + i] = 1.0;
      w[i] = S[(size_t)i * n + i];
    }
    return true;
  }
  Mat A(S);
  return fdtd::la::sym_eig(n, A.data(), Z.data(), w.data());
}

// Z f(w) Z^T
Mat spectral(const Mat& Z, const std::vector<double>& f, int n) {
  Mat T((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[(size_t)i * n + j] = Z[(size_t)i * n + j] * f[j];
  return mul(T, tr(Z, n, n), n, n, n);
}

// Daleckii-Krein pull-back of a symmetric matrix function:
// S_bar = Z (D o (Z^T sym(X) Z)) Z^T
Mat dk_pullback(const Mat& Z, const Mat& D, const Mat& X, int n) {
  Mat Xs((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Xs[(size_t)i * n + j] = 0.5 * (X[(size_t)i * n + j] + X[(size_t)j * n + i]);
  const Mat Zt = tr(Z, n, n);
  Mat T = mul(mul(Zt, Xs, n, n, n), Z, n, n, n);
  for (size_t e = 0; e < T.size(); ++e) T[e] *= D[e];
  return mul(mul(Z, T, n, n, n), Zt, n, n, n);
}

// dJ/dR11 of the eq. (27) clip K~_c = R11^{1/2} M g(M^T M) R22^{1/2},
// M = R11^{-1/2} K R22^{-1/2}, g(mu) = min(1, lim/sqrt(mu)), given dJ/dK~_c
// (R22 and K held).  Difference quotients on the spectra:
//   sqrt: 1/(a+b) (a, b the square roots of two eigenvalues),
//   1/sqrt: -1/(ab(a+b)),
//   g: 0 between two unclipped values, -lim/(ab(a+b)) between two clipped
//      ones, (g_i - g_j)/(mu_i - mu_j) across the bound.
bool clip_vjp(const Mat& R11, const Mat& R22, const Mat& K, int q1, int q2, double lim, const Mat& gK, Mat& gR11) {
  Mat Y, Zr, U;
  std::vector<double> nu, w, mu;
  if (!eig(q1, R11, Y, nu) || !eig(q2, R22, Zr, w)) return false;
  std::vector<double> rn(q1), irn(q1), rw(q2), irw(q2);
  for (int i = 0; i < q1; ++i) {
    if (!(nu[i] > 0)) return false;
    rn[i] = std::sqrt(nu[i]);
    irn[i] = 1.0 / rn[i];
  }
  for (int i = 0; i < q2; ++i) {
    if (!(w[i] > 0)) return false;
    rw[i] = std::sqrt(w[i]);
    irw[i] = 1.0 / rw[i];
  }
  const Mat P = spectral(Y, rn, q1), Q = spectral(Y, irn, q1);
  const Mat R22h = spectral(Zr, rw, q2), R22ih = spectral(Zr, irw, q2);
  const Mat M = mul(mul(Q, K, q1, q1, q2), R22ih, q1, q2, q2);
  const Mat Mt = tr(M, q1, q2);
  if (!eig(q2, mul(Mt, M, q2, q1, q2), U, mu)) return false;
  std::vector<double> sq(q2), g(q2);
  std::vector<char> big(q2);
  for (int i = 0; i < q2; ++i) {
    mu[i] = std::max(mu[i], 0.0);
    sq[i] = std::sqrt(mu[i]);
    big[i] = sq[i] > lim;
    g[i] = big[i] ? lim / sq[i] : 1.0;
  }
  Mat Dg((size_t)q2 * q2, 0.0), Dp((size_t)q1 * q1), Dq((size_t)q1 * q1);
  for (int i = 0; i < q2; ++i)
    for (int j = 0; j < q2; ++j) {
      double v = 0;
      if (big[i] && big[j]) v = -lim / (sq[i] * sq[j] * (sq[i] + sq[j]));
      else if (big[i] != big[j] && mu[i] != mu[j]) v = (g[i] - g[j]) / (mu[i] - mu[j]);
      Dg[(size_t)i * q2 + j] = v;
    }
  for (int i = 0; i < q1; ++i)
    for (int j = 0; j < q1; ++j) {
      Dp[(size_t)i * q1 + j] = 1.0 / (rn[i] + rn[j]);
      Dq[(size_t)i * q1 + j] = -1.0 / (rn[i] * rn[j] * (rn[i] + rn[j]));
    }
  const Mat Gm = spectral(U, g, q2);
  const Mat Phi = mul(M, Gm, q1, q2, q2);
  const Mat gKR = mul(gK, R22h, q1, q2, q2);
  const Mat gP = mul(gKR, tr(Phi, q1, q2), q1, q2, q1);
  const Mat gPhi = mul(P, gKR, q1, q1, q2);
  Mat gM = mul(gPhi, Gm, q1, q2, q2);
  const Mat gS = dk_pullback(U, Dg, mul(Mt, gPhi, q2, q1, q2), q2);
  Mat gS2((size_t)q2 * q2);
  for (int i = 0; i < q2; ++i)
    for (int j = 0; j < q2; ++j) gS2[(size_t)i * q2 + j] = gS[(size_t)i * q2 + j] + gS[(size_t)j * q2 + i];
  const Mat MgS = mul(M, gS2, q1, q2, q2);
  for (size_t e = 0; e < gM.size(); ++e) gM[e] += MgS[e];
  const Mat gQ = mul(mul(gM, R22ih, q1, q2, q2), tr(K, q1, q2), q1, q2, q1);
  const Mat a = dk_pullback(Y, Dp, gP, q1), b = dk_pullback(Y, Dq, gQ, q1);
  gR11.resize((size_t)q1 * q1);
  for (size_t e = 0; e < gR11.size(); ++e) gR11[e] = a[e] + b[e];
  return true;
}

}  // namespace

// What the builder's gradient needs of one build: the build state (fine
// model, E basis, K~ before the clip, the clip's limit), R~ and the sizes.
struct fdtd_rom_model_state {
  BuildState bs;
  Mat Rt;
  double dt = 0;
  size_t nfine = 0;
};

namespace {

// Build with the state kept (as fdtd_rom_build; Rt/Ft/Lt may be null to
// only keep the state).
int build_keep(const fdtd_rom_build_params* prm, fdtd_rom_model_state& st, double* Rt, double* Ft, double* Lt,
               fdtd_rom_build_info* info_out) {
  fdtd_rom_build_info info{};
  if (int rc = build_impl(prm, nullptr, nullptr, nullptr, &info, nullptr); rc != FDTD_OK) return rc;
  const int q = info.q1 + info.q2;
  const int np = 2 * (prm->ni + prm->nj);
  st.Rt.assign((size_t)q * q, 0.0);
  Mat f((size_t)q * q), l((size_t)q * np);
  if (int rc = build_impl(prm, st.Rt.data(), f.data(), l.data(), &info, &st.bs); rc != FDTD_OK) return rc;
  st.dt = prm->dt;
  st.nfine = (size_t)prm->r * prm->ni * prm->r * prm->nj;
  if (Rt) std::copy(st.Rt.begin(), st.Rt.end(), Rt);
  if (Ft) std::copy(f.begin(), f.end(), Ft);
  if (Lt) std::copy(l.begin(), l.end(), Lt);
  if (info_out) *info_out = info;
  return FDTD_OK;
}

// dJ/dR~, dJ/dF~ -> fine-cell dJ/deps_r, dJ/dsigma with the state's basis
int vjp_from_state(const fdtd_rom_model_state& st, const double* grad_Rt, const double* grad_Ft, double* grad_eps_r,
                   double* grad_sigma) {
  const int q1 = st.bs.q1, q2 = st.bs.q2, q = q1 + q2;
  const double dt = st.dt;
  // the E block of dJ/dR~ (through the clip when it acted) and of dJ/dF~
  Mat gR11((size_t)q1 * q1), gF11((size_t)q1 * q1);
  for (int a = 0; a < q1; ++a)
    for (int b = 0; b < q1; ++b) {
      gR11[(size_t)a * q1 + b] = grad_Rt[(size_t)a * q + b];
      gF11[(size_t)a * q1 + b] = grad_Ft[(size_t)a * q + b];
    }
  if (st.bs.clipped) {
    // R~12 = -K~_c/2, R~21 = -K~_c^T/2, F~12 = -K~_c/2, F~21 = +K~_c^T/2
    Mat gK((size_t)q1 * q2), R11((size_t)q1 * q1), R22((size_t)q2 * q2), g;
    for (int a = 0; a < q1; ++a)
      for (int c = 0; c < q2; ++c)
        gK[(size_t)a * q2 + c] = -0.5 * grad_Rt[(size_t)a * q + q1 + c] - 0.5 * grad_Rt[(size_t)(q1 + c) * q + a] -
                                 0.5 * grad_Ft[(size_t)a * q + q1 + c] + 0.5 * grad_Ft[(size_t)(q1 + c) * q + a];
    for (int a = 0; a < q1; ++a)
      for (int b = 0; b < q1; ++b) R11[(size_t)a * q1 + b] = dt * st.Rt[(size_t)a * q + b];
    for (int a = 0; a < q2; ++a)
      for (int b = 0; b < q2; ++b) R22[(size_t)a * q2 + b] = dt * st.Rt[(size_t)(q1 + a) * q + q1 + b];
    if (!clip_vjp(R11, R22, st.bs.K0, q1, q2, st.bs.lim, gK, g))
      return fail(FDTD_EINVAL, "eigen-decomposition for the clip's gradient did not converge");
    for (size_t e = 0; e < gR11.size(); ++e) gR11[e] += dt * g[e];
  }
  // congruence: per E coordinate e, dJ/dDe = (V1 gR11 V1^T)_ee / dt,
  // dJ/dDs = (V1 gF11 V1^T)_ee / 2 (V1 = I for the identity basis)
  const FineModel& fm = st.bs.fm;
  const size_t nf = st.nfine;
  std::fill(grad_eps_r, grad_eps_r + nf, 0.0);
  std::fill(grad_sigma, grad_sigma + nf, 0.0);
  const bool ident = st.bs.V1.empty();
  std::vector<double> u(q1), tR(q1), tF(q1);
  for (int e = 0; e < fm.nE; ++e) {
    double dDe, dDs;
    if (ident) {
      dDe = gR11[(size_t)e * q1 + e] / dt;
      dDs = 0.5 * gF11[(size_t)e * q1 + e];
    } else {
      for (int a = 0; a < q1; ++a) u[a] = st.bs.V1[a][e];
      std::fill(tR.begin(), tR.end(), 0.0);
      std::fill(tF.begin(), tF.end(), 0.0);
      for (int a = 0; a < q1; ++a) {
        if (u[a] == 0.0) continue;
        fdtd::la::axpy(u[a], gR11.data() + (size_t)a * q1, tR.data(), q1);
        fdtd::la::axpy(u[a], gF11.data() + (size_t)a * q1, tF.data(), q1);
      }
      dDe = fdtd::la::dot(tR.data(), u.data(), q1) / dt;
      dDs = 0.5 * fdtd::la::dot(tF.data(), u.data(), q1);
    }
    for (const auto& cw : fm.ecells[e]) {
      grad_eps_r[cw.first] += cw.second * kEps0 * dDe;
      grad_sigma[cw.first] += cw.second * dDs;
    }
  }
  return FDTD_OK;
}

}  // namespace

extern "C" int fdtd_rom_build_vjp(const fdtd_rom_build_params* prm, const double* grad_Rt, const double* grad_Ft,
                                  double* grad_eps_r, double* grad_sigma) {
  if (!prm || !grad_Rt || !grad_Ft || !grad_eps_r || !grad_sigma) return fail(FDTD_EINVAL, "null argument");
  try {
    fdtd_rom_model_state st;
    if (int rc = build_keep(prm, st, nullptr, nullptr, nullptr, nullptr); rc != FDTD_OK) return rc;
    return vjp_from_state(st, grad_Rt, grad_Ft, grad_eps_r, grad_sigma);
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

extern "C" int fdtd_rom_build_keep(const fdtd_rom_build_params* prm, double* Rt, double* Ft, double* Lt,
                                   fdtd_rom_build_info* info, fdtd_rom_model_state** state) {
  if (!prm || !Rt || !Ft || !Lt || !state) return fail(FDTD_EINVAL, "null argument");
  *state = nullptr;
  try {
    std::unique_ptr<fdtd_rom_model_state> st(new fdtd_rom_model_state());
    if (int rc = build_keep(prm, *st, Rt, Ft, Lt, info); rc != FDTD_OK) return rc;
    *state = st.release();
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

extern "C" int fdtd_rom_model_state_vjp(const fdtd_rom_model_state* state, const double* grad_Rt,
                                        const double* grad_Ft, double* grad_eps_r, double* grad_sigma) {
  if (!state || !grad_Rt || !grad_Ft || !grad_eps_r || !grad_sigma) return fail(FDTD_EINVAL, "null argument");
  try {
    return vjp_from_state(*state, grad_Rt, grad_Ft, grad_eps_r, grad_sigma);
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

extern "C" void fdtd_rom_model_state_free(fdtd_rom_model_state* state) { delete state; }
