// Host runtime of the C ABI declared in include/fdtd_rom.h.
//
// create(): validates the problem (eq. (1) CFL, geometry, eq. (26a)
// passivity by Cholesky), folds the coarse interface half cells of eq. (13)
// into the closed form of eq. (23) in FP64, and lays everything out in the
// caller's device workspace.  run(): per step one fused stencil launch and
// one coupling launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/fdtd_rom.h"
#include "common.hpp"
#include "linalg.hpp"
#include "runtime.hpp"

using namespace fdtd;

namespace {
thread_local std::string g_err;
}  // namespace

int fdtd::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Shape-level validation and workspace plan (no numerics).
int fdtd::plan_problem(const fdtd_problem* p, Layout& L) {
  if (!p) return fail(FDTD_EINVAL, "null problem");
  const fdtd_grid& g = p->grid;
  if (g.nx < 2 || g.ny < 2) return fail(FDTD_EINVAL, "grid must be at least 2x2 (got %dx%d)", g.nx, g.ny);
  if (!(g.dx > 0) || !(g.dy > 0) || !(g.dt > 0)) return fail(FDTD_EINVAL, "dx, dy, dt must be positive");
  if (g.dtype != FDTD_F32 && g.dtype != FDTD_F64) return fail(FDTD_EINVAL, "dtype must be FDTD_F32 or FDTD_F64");
  if (p->max_steps < 1) return fail(FDTD_EINVAL, "max_steps must be >= 1");
  if (p->nroms < 0 || (p->nroms > 0 && !p->roms)) return fail(FDTD_EINVAL, "bad region list");
  if (p->nsources < 0 || p->nsources > kMaxSrc || (p->nsources > 0 && !p->sources))
    return fail(FDTD_EINVAL, "between 0 and %d sources are supported", kMaxSrc);
  if (p->nprobes < 0 || (p->nprobes > 0 && !p->probes)) return fail(FDTD_EINVAL, "bad probe list");
  const size_t ts = g.dtype == FDTD_F32 ? 4 : 8;
  L.tsize = ts;
  if (g.pitch_pad < 0 || g.pitch_pad > 1024 || g.pitch_pad % kWave != 0)
    return fail(FDTD_EINVAL, "pitch_pad=%d must be a multiple of %d in [0, 1024]", g.pitch_pad, kWave);
  L.pitch = (int)align_up((size_t)g.nx, kWave) + g.pitch_pad;
  L.field_elems = (size_t)g.ny * L.pitch;
  // the stencil addresses every field with 32-bit byte offsets
  if ((double)L.field_elems * (double)ts >= 2147483648.0)
    return fail(FDTD_EINVAL, "grid %dx%d too large: one field array must stay below 2 GiB", g.nx, g.ny);
  // matrix slots (shared by group)
  L.slot_of_rom.assign(p->nroms, -1);
  L.slot_rep.clear();
  std::vector<int> group_slot;
  std::vector<int> group_id;
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& r = p->roms[k];
    if (r.ni < 1 || r.nj < 1) return fail(FDTD_EINVAL, "region %d: empty footprint", k);
    if (r.q < 1 || r.q > kMaxQ) return fail(FDTD_EINVAL, "region %d: order q=%d outside [1, %d]", k, r.q, kMaxQ);
    if (ports_of(r) > kMaxPorts) return fail(FDTD_EINVAL, "region %d: %d ports exceed %d", k, ports_of(r), kMaxPorts);
    if (align_up((size_t)r.q + ports_of(r), kWave) * (g.dtype == FDTD_F64 ? 8 : 4) > (size_t)kMaxStageBytes)
      return fail(FDTD_EINVAL, "region %d: q + np = %d exceeds the coupling staging (%d bytes)", k,
                  r.q + ports_of(r), kMaxStageBytes);
    if (!r.Rt || !r.Ft || !r.Lt) return fail(FDTD_EINVAL, "region %d: missing matrices", k);
    int slot = -1;
    if (r.group >= 0) {
      for (size_t s = 0; s < group_id.size(); ++s)
        if (group_id[s] == r.group) slot = group_slot[s];
    }
    if (slot < 0) {
      slot = (int)L.slot_rep.size();
      L.slot_rep.push_back(k);
      if (r.group >= 0) {
        group_id.push_back(r.group);
        group_slot.push_back(slot);
      }
    }
    L.slot_of_rom[k] = slot;
  }
  L.slot_off.clear();
  L.slot_members.assign(L.slot_rep.size(), 0);
  for (int k = 0; k < p->nroms; ++k) L.slot_members[L.slot_of_rom[k]]++;
  L.slot_gemm.assign(L.slot_rep.size(), 0);
  L.slot_gt_off.assign(L.slot_rep.size(), 0);
  size_t me = 0;
  for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
    const fdtd_rom& r = p->roms[L.slot_rep[sl]];
    const int np = ports_of(r);
    const size_t ldg = align_up((size_t)r.q + np, kWave);
    L.slot_off.push_back(me);
    me += align_up((size_t)r.q + np, kRowsPerBlock) * ldg;
    me = align_up(me, 64);
    // shared model, FP32, enough copies: MFMA GEMM over the copies
    if (g.dtype == FDTD_F32 && r.group >= 0 && L.slot_members[sl] >= kMinGemmCopies && ldg <= (size_t)kMaxGemmM) {
      L.slot_gemm[sl] = 1;
      L.slot_gt_off[sl] = me;
      me = align_up(me + ldg * ldg, 64);
    }
  }
  L.mats_elems = me;
  L.x_off.clear();
  L.i_off.clear();
  size_t xe = 0, ie = 0;
  L.nrowblocks = 0;
  L.nblocks_mixed = 0;
  L.ncopies = 0;
  L.smem_gemv = L.smem_mixed = 0;
  for (int k = 0; k < p->nroms; ++k) {
    L.x_off.push_back(xe);
    L.i_off.push_back(ie);
    const size_t ldg = align_up((size_t)p->roms[k].q + ports_of(p->roms[k]), kWave);
    xe = align_up(xe + 2 * align_up((size_t)p->roms[k].q, 64), 64);
    ie = align_up(ie + 2 * (size_t)ports_of(p->roms[k]), 64);
    const int rb = (int)(align_up((size_t)p->roms[k].q + ports_of(p->roms[k]), kRowsPerBlock) / kRowsPerBlock);
    L.nrowblocks += rb;
    L.smem_gemv = std::max(L.smem_gemv, ldg * ts);
    if (L.slot_gemm[L.slot_of_rom[k]]) {
      L.ncopies++;
      L.smem_mixed = std::max(L.smem_mixed, ldg * kGemmCopies * ts);
    } else {
      L.nblocks_mixed += rb;
      L.smem_mixed = std::max(L.smem_mixed, ldg * ts);
    }
  }
  for (size_t sl = 0; sl < L.slot_rep.size(); ++sl)
    if (L.slot_gemm[sl]) {
      const fdtd_rom& r = p->roms[L.slot_rep[sl]];
      const size_t ldg = align_up((size_t)r.q + ports_of(r), kWave);
      L.nblocks_mixed += (int)(align_up((L.slot_members[sl] + kGemmCopies - 1) / kGemmCopies, 8) *
                               (ldg / kGemmRowsPerBlock));
    }
  L.xs_elems = xe;
  L.idx_elems = ie;
  size_t o = 0;
  L.off_ctrl = o;
  o = align_up(o + kCtrlInts * sizeof(int), 256);
  L.off_fields = o;
  o = align_up(o + 6 * L.field_elems * ts, 256);
  L.off_al = o;
  o = align_up(o + L.field_elems * ts, 256);
  L.off_be = o;
  o = align_up(o + L.field_elems * ts, 256);
  L.off_midx = o;
  o = align_up(o + L.field_elems * sizeof(uint16_t), 256);
  L.off_mtab = o;
  o = align_up(o + (size_t)kMaxMaterials * 2 * ts, 256);
  L.off_src = o;
  // at least one (zero) row so unused source slots point at valid memory
  o = align_up(o + (size_t)std::max(p->nsources, 1) * p->max_steps * ts, 256);
  L.off_pbuf = o;
  o = align_up(o + (size_t)p->max_steps * p->nprobes * ts, 256);
  L.off_poff = o;
  o = align_up(o + (size_t)p->nprobes * sizeof(int), 256);
  L.off_pcomp = o;
  o = align_up(o + (size_t)p->nprobes * sizeof(int), 256);
  L.off_roms = o;
  o = align_up(o + (size_t)p->nroms * sizeof(RomDev), 256);
  L.off_blocks = o;
  o = align_up(o + (size_t)L.nrowblocks * sizeof(RowBlock), 256);
  L.off_blocks_mixed = o;
  o = align_up(o + (size_t)L.nblocks_mixed * sizeof(RowBlock), 256);
  L.off_copies = o;
  o = align_up(o + std::max<size_t>(L.ncopies, 1) * sizeof(int), 256);
  L.off_mats = o;
  o = align_up(o + L.mats_elems * ts, 256);
  L.off_xs = o;
  o = align_up(o + L.xs_elems * ts, 256);
  L.off_idx = o;
  o = align_up(o + L.idx_elems * sizeof(int), 256);
  L.off_energy = o;
  o = align_up(o + (size_t)energy_blocks(g.nx, g.ny) * sizeof(double), 256);
  const fdtd_pml& pm = p->pml;
  if (pm.n_xlo < 0 || pm.n_xhi < 0 || pm.n_ylo < 0 || pm.n_yhi < 0)
    return fail(FDTD_EINVAL, "absorbing-layer thicknesses must be >= 0");
  L.pml = (pm.n_xlo | pm.n_xhi | pm.n_ylo | pm.n_yhi) != 0;
  if (L.pml) {
    if (pm.n_xlo + pm.n_xhi >= g.nx || pm.n_ylo + pm.n_yhi >= g.ny)
      return fail(FDTD_EINVAL, "absorbing layers leave no interior cell");
    L.px_stride = (int)align_up((size_t)L.pitch + 1, 64);
    L.py_stride = (int)align_up((size_t)g.ny + 1, 64);
    L.off_prof = o;
    o = align_up(o + 6 * ((size_t)L.px_stride + L.py_stride) * ts, 256);
    L.off_psi = o;
    o = align_up(o + 6 * L.field_elems * ts, 256);
  } else {
    L.tb_ok = true;
    L.max_tiles2 = ((g.nx + kOwned2 - 1) / kOwned2) * ((g.ny + 15) / 16);  // at 4 rows per wave
    L.off_fc = o;
    o = align_up(o + 3 * L.field_elems * ts, 256);
    L.off_role2 = o;
    o = align_up(o + (size_t)L.max_tiles2, 256);
    L.off_near = o;
    o = align_up(o + (size_t)L.max_tiles2 * sizeof(int), 256);
    L.off_st1m = o;
    o = align_up(o + L.field_elems, 256);
  }
  L.total = o;
  return FDTD_OK;
}

namespace {

// Stretched-derivative profiles along one axis of n cells of size d (CPML,
// see fdtd_pml in the header): for E samples k d (k = 0..n) and Hz samples
// (k + 1/2) d (k < n), (1/kappa, b, a), written into out[0..5] at stride S;
// entries past the axis keep the identity (1, 1, 0).
template <typename T>
void pml_axis(int n, double d, double dt, int nlo, int nhi, const fdtd_pml& pm, int S, T* out) {
  const double m = pm.m > 0 ? pm.m : 3.0;
  const double kmax = pm.kappa_max >= 1 ? pm.kappa_max : 1.0;
  const double amax = pm.alpha_max > 0 ? pm.alpha_max : 0.0;
  const double eta0 = kMu0 * kC0;
  const double smax = pm.sigma_scale * 0.8 * (m + 1.0) / (eta0 * d);
  const double len = n * d, dlo = nlo * d, dhi = nhi * d;
  for (int k = 0; k < 6; ++k)
    for (int i = 0; i < S; ++i) out[(size_t)k * S + i] = (T)(k % 3 == 2 ? 0.0 : 1.0);
  auto put = [&](int base, int i, double x) {
    double rho = 0;
    if (nlo > 0 && x < dlo) rho = (dlo - x) / dlo;
    if (nhi > 0 && x > len - dhi) rho = (x - (len - dhi)) / dhi;
    if (!(rho > 0)) return;
    const double pw = std::pow(rho, m);
    const double sigma = smax * pw;
    const double kappa = 1.0 + (kmax - 1.0) * pw;
    const double alpha = amax * (1.0 - rho);
    const double b = std::exp(-(sigma / kappa + alpha) * dt / kEps0);
    const double den = sigma * kappa + kappa * kappa * alpha;
    const double a = sigma > 0 ? sigma * (b - 1.0) / den : 0.0;
    out[(size_t)(base + 0) * S + i] = (T)(1.0 / kappa);
    out[(size_t)(base + 1) * S + i] = (T)b;
    out[(size_t)(base + 2) * S + i] = (T)a;
  };
  for (int i = 0; i <= n; ++i) put(0, i, i * d);
  for (int i = 0; i < n; ++i) put(3, i, (i + 0.5) * d);
}


// Every GEMV row block of a model stages the same inputs (its reduced state
// and the ring Hz, scattered loads from the step-n fields).  Reorder
// v[start, end) so that a model's blocks sit at indices equal modulo 8 -
// workgroup i runs on XCD i % 8, so they share one L2 - as far as the
// counts allow: models go to residues largest first, each to the residue
// with the most free slots; a slot whose residue has run out takes a block
// of another.  Only the order changes (each block is independent).
void xcd_group(std::vector<RowBlock>& v, size_t start) {
  if (v.size() <= start + 8) return;
  std::vector<std::vector<RowBlock>> by_model;
  std::vector<int> slot_of;  // model -> index in by_model
  for (size_t i = start; i < v.size(); ++i) {
    const int k = v[i].a;
    if (k >= (int)slot_of.size()) slot_of.resize(k + 1, -1);
    if (slot_of[k] < 0) {
      slot_of[k] = (int)by_model.size();
      by_model.emplace_back();
    }
    by_model[slot_of[k]].push_back(v[i]);
  }
  std::vector<size_t> order(by_model.size());
  for (size_t m = 0; m < order.size(); ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t a, size_t b) { return by_model[a].size() > by_model[b].size(); });
  long cap[8] = {0};
  for (size_t i = start; i < v.size(); ++i) cap[i % 8]++;
  std::vector<RowBlock> q[8];
  for (size_t m : order) {
    int best = 0;
    for (int r = 1; r < 8; ++r)
      if (cap[r] > cap[best]) best = r;
    cap[best] -= (long)by_model[m].size();
    q[best].insert(q[best].end(), by_model[m].begin(), by_model[m].end());
  }
  size_t head[8] = {0};
  for (size_t i = start; i < v.size(); ++i) {
    int r = (int)(i % 8);
    if (head[r] == q[r].size()) {  // this residue ran out: the fullest other
      int best = -1;
      for (int s = 0; s < 8; ++s)
        if (head[s] < q[s].size() && (best < 0 || q[s].size() - head[s] > q[best].size() - head[best])) best = s;
      r = best;
    }
    v[i] = q[r][head[r]++];
  }
}

template <typename T>
int setup_device(fdtd_rom_sim* s, const fdtd_problem* p, const std::vector<unsigned char>& inside) {
  const Layout& L = s->L;
  const int nx = s->nx, ny = s->ny, P = L.pitch;
  const size_t fe = L.field_elems;
  const fdtd_grid& g = p->grid;
  std::vector<T> host(fe, T(0));
  char* ws = s->ws;
  hipStream_t st = s->stream;
  auto up = [&](size_t off, const void* src, size_t bytes) -> int {
    if (bytes == 0) return FDTD_OK;
    if (hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(FDTD_EDEVICE, "hipMemcpyAsync failed");
    if (hipStreamSynchronize(st) != hipSuccess) return fail(FDTD_EDEVICE, "hipStreamSynchronize failed");
    return FDTD_OK;
  };
  int rc;
  // control block
  int ctrl[kCtrlInts] = {0, 0, 0, 0};
  if ((rc = up(L.off_ctrl, ctrl, sizeof(ctrl))) != FDTD_OK) return rc;
  // fields: Hz zero; E zero except the interface value L~^T x0 of each region
  std::vector<T> ex(fe, T(0)), ey(fe, T(0));
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& r = p->roms[k];
    if (!r.x0) continue;
    const int np = ports_of(r);
    for (int c = 0; c < np; ++c) {
      double y = 0;
      for (int a = 0; a < r.q; ++a) y += r.Lt[(size_t)a * np + c] * r.x0[a];
      int ei, ej;
      bool isx;
      if (c < r.ni) { ei = r.i0 + c; ej = r.j0; isx = true; }
      else if (c < 2 * r.ni) { ei = r.i0 + c - r.ni; ej = r.j0 + r.nj; isx = true; }
      else if (c < 2 * r.ni + r.nj) { ei = r.i0; ej = r.j0 + c - 2 * r.ni; isx = false; }
      else { ei = r.i0 + r.ni; ej = r.j0 + c - 2 * r.ni - r.nj; isx = false; }
      (isx ? ex : ey)[(size_t)ej * P + ei] = (T)y;
    }
  }
  const size_t fb = fe * sizeof(T);
  for (int set = 0; set < 2; ++set) {
    if ((rc = up(L.off_fields + (3 * set + 0) * fb, host.data(), fb)) != FDTD_OK) return rc;
    if ((rc = up(L.off_fields + (3 * set + 1) * fb, ex.data(), fb)) != FDTD_OK) return rc;
    if ((rc = up(L.off_fields + (3 * set + 2) * fb, ey.data(), fb)) != FDTD_OK) return rc;
  }
  if (L.tb_ok) {  // the two-step launches' step-(n+1) set starts as a copy of the state
    if ((rc = up(L.off_fc, host.data(), fb)) != FDTD_OK) return rc;
    if ((rc = up(L.off_fc + fb, ex.data(), fb)) != FDTD_OK) return rc;
    if ((rc = up(L.off_fc + 2 * fb, ey.data(), fb)) != FDTD_OK) return rc;
  }
  // per-cell material: a = eps0*eps_r/dt (negative inside regions, zero on
  // PEC cells: the stencil then never updates the cell's Hz or its edges,
  // as for the padding columns), b = sigma/2
  std::vector<T> al(fe, T(0)), be(fe, T(0));
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)j * nx + i;
      const double er = g.eps_r ? g.eps_r[c] : 1.0;
      const double sg = g.sigma ? g.sigma[c] : 0.0;
      const bool metal = g.pec && g.pec[c];
      al[(size_t)j * P + i] = inside[c] ? T(-1) : metal ? T(0) : (T)(kEps0 * er / g.dt);
      be[(size_t)j * P + i] = (inside[c] || metal) ? T(0) : (T)(sg / 2.0);
    }
  if ((rc = up(L.off_al, al.data(), fb)) != FDTD_OK) return rc;
  if ((rc = up(L.off_be, be.data(), fb)) != FDTD_OK) return rc;
  if (L.tb_ok) {
    // where the second launch of a pair reads the step-(n+1) set: the box
    // x in [i-1, i+2], y in [j-1, j+2] around each ring cell (i, j) (the
    // band's Hz and edges and the ring gathers, each Hz formed from its
    // cell, the Ex above and the Ey east of it)
    std::vector<uint8_t> m(fe, 0);
    for (int k = 0; k < p->nroms; ++k) {
      const fdtd_rom& r = p->roms[k];
      const int np = ports_of(r);
      for (int c = 0; c < np; ++c) {
        int oi, oj;
        if (c < r.ni) { oi = r.i0 + c; oj = r.j0 - 1; }
        else if (c < 2 * r.ni) { oi = r.i0 + c - r.ni; oj = r.j0 + r.nj; }
        else if (c < 2 * r.ni + r.nj) { oi = r.i0 - 1; oj = r.j0 + c - 2 * r.ni; }
        else { oi = r.i0 + r.ni; oj = r.j0 + c - 2 * r.ni - r.nj; }
        for (int dy = -1; dy <= 2; ++dy)
          for (int dx = -1; dx <= 2; ++dx) {
            const int i = oi + dx, j = oj + dy;
            if (i >= 0 && i < nx && j >= 0 && j < ny) m[(size_t)j * P + i] = 1;
          }
      }
    }
    if ((rc = up(L.off_st1m, m.data(), fe)) != FDTD_OK) return rc;
  }
  // the same material as a 16-bit index into a table of the distinct (a, b)
  // pairs (exact bit patterns), when there are at most kMaxMaterials of them
  {
    struct Key {
      uint64_t a, b;
      bool operator==(const Key& o) const { return a == o.a && b == o.b; }
    };
    struct KeyHash {
      size_t operator()(const Key& k) const {
        return (size_t)(k.a * 0x9E3779B97F4A7C15ull ^ (k.b + 0x632BE59BD9B4E019ull + (k.a << 6) + (k.a >> 2)));
      }
    };
    auto bits = [](T v) {
      uint64_t u = 0;
      std::memcpy(&u, &v, sizeof(T));
      return u;
    };
    std::unordered_map<Key, uint16_t, KeyHash> ids;
    std::vector<uint16_t> mid(fe);
    std::vector<MatPair<T>> tab;
    bool fits = true;
    Key last{~0ull, ~0ull};
    uint16_t last_id = 0;
    for (size_t k = 0; k < fe && fits; ++k) {
      const Key key{bits(al[k]), bits(be[k])};
      if (!(key == last)) {
        auto it = ids.find(key);
        if (it == ids.end()) {
          if (tab.size() == (size_t)kMaxMaterials) {
            fits = false;
            break;
          }
          it = ids.emplace(key, (uint16_t)tab.size()).first;
          tab.push_back(MatPair<T>{al[k], be[k]});
        }
        last = key;
        last_id = it->second;
      }
      mid[k] = last_id;
    }
    s->nmat = fits ? (int)tab.size() : 0;
    if (fits) {
      if ((rc = up(L.off_midx, mid.data(), fe * sizeof(uint16_t))) != FDTD_OK) return rc;
      if ((rc = up(L.off_mtab, tab.data(), tab.size() * sizeof(MatPair<T>))) != FDTD_OK) return rc;
    }
  }
  // sources
  std::vector<T> sv((size_t)std::max(p->nsources, 1) * p->max_steps, T(0));
  for (int k = 0; k < p->nsources; ++k)
    for (int n = 0; n < p->max_steps; ++n)
      sv[(size_t)k * p->max_steps + n] = (T)p->sources[k].incr[n];
  if ((rc = up(L.off_src, sv.data(), sv.size() * sizeof(T))) != FDTD_OK) return rc;
  // probes
  std::vector<int> poff(p->nprobes), pcomp(p->nprobes);
  for (int k = 0; k < p->nprobes; ++k) {
    poff[k] = p->probes[k].j * P + p->probes[k].i;
    pcomp[k] = p->probes[k].comp;
  }
  if ((rc = up(L.off_poff, poff.data(), poff.size() * sizeof(int))) != FDTD_OK) return rc;
  if ((rc = up(L.off_pcomp, pcomp.data(), pcomp.size() * sizeof(int))) != FDTD_OK) return rc;
  std::vector<T> zeros_pbuf((size_t)p->max_steps * p->nprobes, T(0));
  if ((rc = up(L.off_pbuf, zeros_pbuf.data(), zeros_pbuf.size() * sizeof(T))) != FDTD_OK) return rc;
  // regions
  std::vector<RomDev> rd(p->nroms);
  std::vector<T> mats(L.mats_elems, T(0));
  std::vector<T> xs(L.xs_elems, T(0));
  std::vector<int> idx(L.idx_elems, 0);
  // G = [[A~, B~'], [C~ A~, C~ B~']] (eq. (23) on [x~^n; h]), row-major,
  // rows padded to kRowsPerBlock, row length padded to a multiple of 64
  for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
    const RomHost& h = s->roms[L.slot_rep[sl]];
    const int q = h.q, np = h.np, nc = q + np;
    const size_t ldg = align_up((size_t)nc, kWave);
    T* g = mats.data() + L.slot_off[sl];
    std::vector<double> CA((size_t)np * q), CB((size_t)np * np);
    la::gemm(np, q, q, h.C.data(), h.A.data(), CA.data());
    la::gemm(np, np, q, h.C.data(), h.B.data(), CB.data());
    for (int a = 0; a < q; ++a) {
      for (int c = 0; c < q; ++c) g[(size_t)a * ldg + c] = (T)h.A[(size_t)a * q + c];
      for (int c = 0; c < np; ++c) g[(size_t)a * ldg + q + c] = (T)h.B[(size_t)a * np + c];
    }
    for (int k = 0; k < np; ++k) {
      for (int c = 0; c < q; ++c) g[(size_t)(q + k) * ldg + c] = (T)CA[(size_t)k * q + c];
      for (int c = 0; c < np; ++c) g[(size_t)(q + k) * ldg + q + c] = (T)CB[(size_t)k * np + c];
    }
  }
  for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
    if (!L.slot_gemm[sl]) continue;
    const RomHost& h = s->roms[L.slot_rep[sl]];
    const size_t ldg = align_up((size_t)h.q + h.np, kWave);
    const T* g = mats.data() + L.slot_off[sl];
    T* gt = mats.data() + L.slot_gt_off[sl];
    for (size_t a = 0; a < ldg && a < align_up((size_t)h.q + h.np, kRowsPerBlock); ++a)
      for (size_t c = 0; c < ldg; ++c) gt[c * ldg + a] = g[a * ldg + c];
  }
  std::vector<RowBlock> blocks, mixed;
  std::vector<int> copies;
  for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
    if (!L.slot_gemm[sl]) continue;
    std::vector<int> members;
    for (int k = 0; k < p->nroms; ++k)
      if (L.slot_of_rom[k] == (int)sl) members.push_back(k);
    const fdtd_rom& rr = p->roms[L.slot_rep[sl]];
    const int ldg = (int)align_up((size_t)rr.q + ports_of(rr), kWave);
    // Every row block of a group of copies gathers that group's inputs (its
    // reduced states and the ring Hz, scattered loads from the step-n
    // fields).  Blocks are listed row block by row block over the groups,
    // the groups padded to a multiple of 8 with empty blocks, so that a
    // group's row blocks sit at workgroup indices equal modulo 8: the same
    // XCD, whose L2 then serves the repeated gathers (they were spread over
    // four XCDs).
    const size_t first = copies.size();
    const size_t ngroups = (members.size() + kGemmCopies - 1) / kGemmCopies;
    for (size_t c = 0; c < members.size(); ++c) copies.push_back(members[c]);
    for (int row0 = 0; row0 < ldg; row0 += kGemmRowsPerBlock)
      for (size_t g = 0; g < align_up(ngroups, 8); ++g) {
        const size_t c0 = g * kGemmCopies;
        const int cnt = g < ngroups ? (int)std::min<size_t>(kGemmCopies, members.size() - c0) : 0;
        // an empty block points at the group's first copy (a valid
        // descriptor) and writes nothing
        mixed.push_back(RowBlock{1, row0 / 16, (int)(first + (g < ngroups ? c0 : 0)), cnt});
      }
  }
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& r = p->roms[k];
    const int np = ports_of(r);
    rd[k].q = r.q;
    rd[k].np = np;
    rd[k].n_ex = 2 * r.ni;
    rd[k].ldg = (int)align_up((size_t)r.q + np, kWave);
    rd[k].g_off = (int64_t)L.slot_off[L.slot_of_rom[k]];
    rd[k].x_off = (int64_t)L.x_off[k];
    rd[k].xstride = (int64_t)align_up((size_t)r.q, 64);
    rd[k].i_off = (int64_t)L.i_off[k];
    rd[k].gt_off = L.slot_gemm[L.slot_of_rom[k]] ? (int64_t)L.slot_gt_off[L.slot_of_rom[k]] : -1;
    for (int row0 = 0; row0 < r.q + np; row0 += kRowsPerBlock) {
      blocks.push_back(RowBlock{0, k, row0, 0});
      if (!L.slot_gemm[L.slot_of_rom[k]]) mixed.push_back(RowBlock{0, k, row0, 0});
    }
    if (r.x0)
      for (int a = 0; a < r.q; ++a) xs[L.x_off[k] + a] = (T)r.x0[a];
    int* gi = idx.data() + L.i_off[k];
    int* si = gi + np;
    for (int c = 0; c < np; ++c) {
      int ei, ej, oi, oj;
      if (c < r.ni) { ei = r.i0 + c; ej = r.j0; oi = ei; oj = r.j0 - 1; }
      else if (c < 2 * r.ni) { ei = r.i0 + c - r.ni; ej = r.j0 + r.nj; oi = ei; oj = ej; }
      else if (c < 2 * r.ni + r.nj) { ei = r.i0; ej = r.j0 + c - 2 * r.ni; oi = r.i0 - 1; oj = ej; }
      else { ei = r.i0 + r.ni; ej = r.j0 + c - 2 * r.ni - r.nj; oi = ei; oj = ej; }
      gi[c] = oj * P + oi;
      si[c] = ej * P + ei;
    }
  }
  if ((int)blocks.size() != L.nrowblocks || (int)mixed.size() != L.nblocks_mixed || copies.size() != L.ncopies)
    return fail(FDTD_EINVAL, "internal: coupling block count mismatch");
  // GEMV blocks (after the GEMM blocks, whose count is a multiple of 8) in
  // XCD groups per model
  {
    size_t ngemm = 0;
    while (ngemm < mixed.size() && mixed[ngemm].kind == 1) ++ngemm;
    xcd_group(blocks, 0);
    xcd_group(mixed, ngemm);
  }
  if ((rc = up(L.off_blocks, blocks.data(), blocks.size() * sizeof(RowBlock))) != FDTD_OK) return rc;
  if ((rc = up(L.off_blocks_mixed, mixed.data(), mixed.size() * sizeof(RowBlock))) != FDTD_OK) return rc;
  if ((rc = up(L.off_copies, copies.data(), copies.size() * sizeof(int))) != FDTD_OK) return rc;
  if ((rc = up(L.off_roms, rd.data(), rd.size() * sizeof(RomDev))) != FDTD_OK) return rc;
  if ((rc = up(L.off_mats, mats.data(), mats.size() * sizeof(T))) != FDTD_OK) return rc;
  if ((rc = up(L.off_xs, xs.data(), xs.size() * sizeof(T))) != FDTD_OK) return rc;
  if ((rc = up(L.off_idx, idx.data(), idx.size() * sizeof(int))) != FDTD_OK) return rc;

  // kernel parameter block
  StepParams<T> sp{};
  for (int set = 0; set < 2; ++set)
    for (int c = 0; c < 3; ++c) sp.f[set][c] = (T*)(ws + L.off_fields + (3 * set + c) * fb);
  sp.al = (const T*)(ws + L.off_al);
  sp.be = (const T*)(ws + L.off_be);
  sp.mi = (const uint16_t*)(ws + L.off_midx);
  sp.mt = (const MatPair<T>*)(ws + L.off_mtab);
  sp.midx = s->nmat > 0 ? 1 : 0;
  sp.ctrl = (int*)(ws + L.off_ctrl);
  sp.step_off = 0;
  sp.nx = nx;
  sp.ny = ny;
  sp.pitch = P;
  sp.tiles_x = (nx + kWave - 1) / kWave;
  sp.nst_blocks = 0;  // set per tiling in set_tiling()
  sp.chdy = (T)(g.dt / (kMu0 * g.dy));
  sp.chdx = (T)(g.dt / (kMu0 * g.dx));
  sp.k2dy = (T)(2.0 / g.dy);
  sp.k2dx = (T)(2.0 / g.dx);
  sp.nsrc = p->nsources;
  for (int k = 0; k < kMaxSrc; ++k) {
    sp.src[k].comp = -1;
    sp.src[k].incr = (const T*)(ws + L.off_src);
  }
  for (int k = 0; k < p->nsources; ++k) {
    const fdtd_source& so = p->sources[k];
    sp.src[k].comp = so.comp;
    sp.src[k].i0 = so.i0;
    sp.src[k].i1 = so.i1;
    sp.src[k].j0 = so.j0;
    sp.src[k].j1 = so.j1;
    sp.src[k].incr = (const T*)(ws + L.off_src) + (size_t)k * p->max_steps;
  }
  sp.roms = (const RomDev*)(ws + L.off_roms);
  sp.copies = (const int*)(ws + L.off_copies);
  // shared groups use the MFMA GEMM when eligible (fdtd_rom_set_shared_gemm)
  sp.blocks = (const RowBlock*)(ws + L.off_blocks_mixed);
  sp.nrowblocks = L.nblocks_mixed;
  sp.ncoup_blocks = (L.nblocks_mixed + 7) / 8 * 8;
  s->smem = L.smem_mixed;
  sp.mats = (const T*)(ws + L.off_mats);
  sp.xs = (T*)(ws + L.off_xs);
  sp.idx = (const int*)(ws + L.off_idx);
  sp.nprobes = p->nprobes;
  sp.probe_off = (const int*)(ws + L.off_poff);
  sp.probe_comp = (const int*)(ws + L.off_pcomp);
  sp.probe_buf = (T*)(ws + L.off_pbuf);
  // absorbing layers
  sp.pml = L.pml ? 1 : 0;
  sp.pml_xlo = p->pml.n_xlo;
  sp.pml_xhi = p->pml.n_xhi;
  sp.pml_ylo = p->pml.n_ylo;
  sp.pml_yhi = p->pml.n_yhi;
  sp.px_stride = L.px_stride;
  sp.py_stride = L.py_stride;
  if (L.pml) {
    std::vector<T> prof(6 * ((size_t)L.px_stride + L.py_stride));
    pml_axis<T>(nx, g.dx, g.dt, p->pml.n_xlo, p->pml.n_xhi, p->pml, L.px_stride, prof.data());
    pml_axis<T>(ny, g.dy, g.dt, p->pml.n_ylo, p->pml.n_yhi, p->pml, L.py_stride,
                prof.data() + 6 * (size_t)L.px_stride);
    if ((rc = up(L.off_prof, prof.data(), prof.size() * sizeof(T))) != FDTD_OK) return rc;
    if (hipMemsetAsync(ws + L.off_psi, 0, 6 * fb, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return fail(FDTD_EDEVICE, "hipMemsetAsync failed");
    sp.px = (const T*)(ws + L.off_prof);
    sp.py = sp.px + 6 * (size_t)L.px_stride;
    T* ps = (T*)(ws + L.off_psi);
    sp.psi_h[0][0] = ps;
    sp.psi_h[0][1] = ps + fe;
    sp.psi_h[1][0] = ps + 2 * fe;
    sp.psi_h[1][1] = ps + 3 * fe;
    sp.psi_ex = ps + 4 * fe;
    sp.psi_ey = ps + 5 * fe;
  }
  if constexpr (sizeof(T) == 4) s->sp_f = sp;
  else s->sp_d = sp;
  return FDTD_OK;
}

// RHS <- M^{-1} RHS (q x (q + np)).  When M = [[D1, M12], [0, D2]] with D1
// and D2 diagonal (a model kept in the identity basis: R~ + F~ is block
// upper triangular and its diagonal blocks are diagonal, the interface
// terms L~ C+ L~^T touch distinct port rows), block back substitution
// X2 = D2^{-1} RHS2, X1 = D1^{-1} (RHS1 - M12 X2) with one threaded product;
// otherwise LU with partial pivoting.  False if M is singular.
bool solve_closed_form(int q, int np, std::vector<double>& M, std::vector<double>& RHS) {
  const int m = q + np;
  auto diag_only = [&](int r, int c0, int c1) {
    for (int c = c0; c < c1; ++c)
      if (c != r && M[(size_t)r * q + c] != 0.0) return false;
    return M[(size_t)r * q + r] != 0.0;
  };
  int t = 0;  // trailing rows with only their diagonal
  while (t < q && diag_only(q - 1 - t, 0, q)) ++t;
  const int q1 = q - t;
  bool structured = t > 0 && q1 > 0;
  for (int r = 0; r < q1 && structured; ++r) structured = diag_only(r, 0, q1);
  if (!structured) {
    std::vector<int> piv;
    if (!la::lu_factor(q, M.data(), piv)) return false;
    la::lu_solve(q, M.data(), piv, RHS.data(), m);
    return true;
  }
  for (int r = q1; r < q; ++r) {
    const double inv = 1.0 / M[(size_t)r * q + r];
    for (int c = 0; c < m; ++c) RHS[(size_t)r * m + c] *= inv;
  }
  // P = M12 X2 as C[i][j] = dot(M12 row i, X2 column j)
  std::vector<std::vector<double>> X2t(m, std::vector<double>(t));
  for (int r = 0; r < t; ++r)
    for (int c = 0; c < m; ++c) X2t[c][r] = RHS[(size_t)(q1 + r) * m + c];
  std::vector<const double*> Ap(q1), Bp(m);
  for (int r = 0; r < q1; ++r) Ap[r] = M.data() + (size_t)r * q + q1;
  for (int c = 0; c < m; ++c) Bp[c] = X2t[c].data();
  std::vector<double> Pm((size_t)q1 * m);
  la::gram_mt(Ap.data(), q1, Bp.data(), m, (size_t)t, Pm.data(), m);
  for (int r = 0; r < q1; ++r) {
    const double inv = 1.0 / M[(size_t)r * q + r];
    for (int c = 0; c < m; ++c) RHS[(size_t)r * m + c] = (RHS[(size_t)r * m + c] - Pm[(size_t)r * m + c]) * inv;
  }
  return true;
}

// Is the symmetric q x q matrix A positive definite?  With A = [D B; B^T C]
// and D its largest leading diagonal block (the whole E block of a model
// kept in the identity basis), A > 0 exactly when D > 0 and the Schur
// complement C - B^T D^{-1} B > 0 (checked by Cholesky); with no diagonal
// leading block this is a Cholesky of A itself.
bool positive_definite(int q, const double* A) {
  int k = 0;
  for (; k < q; ++k) {
    bool diag_row = true;
    for (int b = 0; b < k && diag_row; ++b) diag_row = A[(size_t)k * q + b] == 0.0;
    if (!diag_row || !(A[(size_t)k * q + k] > 0.0)) break;
  }
  const int m = q - k;
  if (m == 0) return true;
  // rows of D^{-1/2} B as columns: Bt[c][a] = A[a][k + c] / sqrt(A[a][a])
  std::vector<std::vector<double>> Bt(m, std::vector<double>(k));
  for (int a = 0; a < k; ++a) {
    const double s = 1.0 / std::sqrt(A[(size_t)a * q + a]);
    for (int c = 0; c < m; ++c) Bt[c][a] = A[(size_t)a * q + k + c] * s;
  }
  std::vector<const double*> Bp(m);
  for (int c = 0; c < m; ++c) Bp[c] = Bt[c].data();
  std::vector<double> S((size_t)m * m, 0.0);
  if (k > 0) la::gram_mt(Bp.data(), m, Bp.data(), m, (size_t)k, S.data(), m, true);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b <= a; ++b) S[(size_t)a * m + b] = A[(size_t)(k + a) * q + k + b] - S[(size_t)a * m + b];
  return la::cholesky(m, S.data());
}

int coupling_precompute(const fdtd_problem* p, std::vector<RomHost>& out) {
  const fdtd_grid& g = p->grid;
  const int nx = g.nx;
  out.resize(p->nroms);
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& r = p->roms[k];
    RomHost& h = out[k];
    h.i0 = r.i0; h.j0 = r.j0; h.ni = r.ni; h.nj = r.nj; h.q = r.q;
    const int q = r.q, np = ports_of(r);
    h.np = np;
    // eq. (26a): R~ symmetric positive definite
    double rmax = 0, asym = 0;
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        rmax = std::max(rmax, std::fabs(r.Rt[(size_t)a * q + b]));
        asym = std::max(asym, std::fabs(r.Rt[(size_t)a * q + b] - r.Rt[(size_t)b * q + a]));
      }
    if (!(asym <= 1e-12 * rmax))
      return fail(FDTD_ENOTPASSIVE, "region %d: R~ not symmetric (%.3g relative)", k, asym / rmax);
    if (!positive_definite(q, r.Rt))
      return fail(FDTD_ENOTPASSIVE, "region %d: R~ is not positive definite at dt (eq. 26a)", k);
    // coarse half cells of eq. (13): Dl Dl' (eps/dt +- sigma/2), outside material
    std::vector<double> cp(np), cm(np), sc(np);
    for (int c = 0; c < np; ++c) {
      int oi, oj;
      double dl, dlh, s;
      if (c < r.ni) { oi = r.i0 + c; oj = r.j0 - 1; dl = g.dx; dlh = g.dy / 2; s = -g.dx; }
      else if (c < 2 * r.ni) { oi = r.i0 + c - r.ni; oj = r.j0 + r.nj; dl = g.dx; dlh = g.dy / 2; s = g.dx; }
      else if (c < 2 * r.ni + r.nj) { oi = r.i0 - 1; oj = r.j0 + c - 2 * r.ni; dl = g.dy; dlh = g.dx / 2; s = g.dy; }
      else { oi = r.i0 + r.ni; oj = r.j0 + c - 2 * r.ni - r.nj; dl = g.dy; dlh = g.dx / 2; s = -g.dy; }
      const size_t ci = (size_t)oj * nx + oi;
      const double e = kEps0 * (g.eps_r ? g.eps_r[ci] : 1.0);
      const double sg = g.sigma ? g.sigma[ci] : 0.0;
      cp[c] = dl * dlh * (e / g.dt + sg / 2.0);
      cm[c] = dl * dlh * (e / g.dt - sg / 2.0);
      sc[c] = s;
    }
    // M = R~ + F~ + L~ C+ L~^T ;  RHS = [R~ - F~ + L~ C- L~^T | L~ Sc]
    // (the L~ C L~^T terms summed over the rows of L~ that are not zero)
    std::vector<double> M((size_t)q * q), RHS((size_t)q * (q + np));
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        const double R = r.Rt[(size_t)a * q + b], F = r.Ft[(size_t)a * q + b];
        M[(size_t)a * q + b] = R + F;
        RHS[(size_t)a * (q + np) + b] = R - F;
      }
    std::vector<int> lrows;
    for (int a = 0; a < q; ++a)
      for (int c = 0; c < np; ++c)
        if (r.Lt[(size_t)a * np + c] != 0.0) {
          lrows.push_back(a);
          break;
        }
    for (int a : lrows)
      for (int b : lrows) {
        double sp = 0, sm = 0;
        for (int c = 0; c < np; ++c) {
          const double l = r.Lt[(size_t)a * np + c] * r.Lt[(size_t)b * np + c];
          sp += l * cp[c];
          sm += l * cm[c];
        }
        M[(size_t)a * q + b] += sp;
        RHS[(size_t)a * (q + np) + b] += sm;
      }
    for (int a = 0; a < q; ++a)
      for (int c = 0; c < np; ++c) RHS[(size_t)a * (q + np) + q + c] = r.Lt[(size_t)a * np + c] * sc[c];
    if (!solve_closed_form(q, np, M, RHS))
      return fail(FDTD_ENOTPASSIVE, "region %d: coupled update matrix is singular", k);
    h.A.assign((size_t)q * q, 0.0);
    h.B.assign((size_t)q * np, 0.0);
    h.C.assign((size_t)np * q, 0.0);
    for (int a = 0; a < q; ++a) {
      for (int b = 0; b < q; ++b) h.A[(size_t)a * q + b] = RHS[(size_t)a * (q + np) + b];
      for (int c = 0; c < np; ++c) h.B[(size_t)a * np + c] = RHS[(size_t)a * (q + np) + q + c];
    }
    for (int c = 0; c < np; ++c)
      for (int a = 0; a < q; ++a) h.C[(size_t)c * q + a] = r.Lt[(size_t)a * np + c];
    h.R.assign(r.Rt, r.Rt + (size_t)q * q);
    h.F.assign(r.Ft, r.Ft + (size_t)q * q);
    h.cp = std::move(cp);
    h.cm = std::move(cm);
    h.sc = std::move(sc);
  }
  return FDTD_OK;
}

// Coarse cell just outside port c of region r (the ring cell whose Hz the
// port gathers and whose half cell enters eq. (13)).
struct PortCell {
  int oi, oj;
};
PortCell port_cell(const fdtd_rom& r, int c) {
  if (c < r.ni) return {r.i0 + c, r.j0 - 1};
  if (c < 2 * r.ni) return {r.i0 + c - r.ni, r.j0 + r.nj};
  if (c < 2 * r.ni + r.nj) return {r.i0 - 1, r.j0 + c - 2 * r.ni};
  return {r.i0 + r.ni, r.j0 + c - 2 * r.ni - r.nj};
}

int validate_numbers(const fdtd_problem* p, const Layout& L, std::vector<unsigned char>& inside) {
  const fdtd_grid& g = p->grid;
  const int nx = g.nx, ny = g.ny;
  double emin = 1e300;
  for (size_t c = 0; c < (size_t)nx * ny; ++c) {
    const double e = g.eps_r ? g.eps_r[c] : 1.0;
    const double s = g.sigma ? g.sigma[c] : 0.0;
    if (!(e > 0) || !std::isfinite(e)) return fail(FDTD_EINVAL, "eps_r must be positive and finite");
    if (!(s >= 0) || !std::isfinite(s)) return fail(FDTD_EINVAL, "sigma must be non-negative and finite");
    emin = std::min(emin, e);
  }
  // eq. (1) on the coarse grid, slowest-medium-free bound c = c0/sqrt(min eps_r)
  const double c = kC0 / std::sqrt(emin);
  const double lim = 1.0 / (c * std::sqrt(1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy)));
  if (g.dt > lim) return fail(FDTD_EINVAL, "dt=%.6g exceeds the coarse CFL limit %.6g of eq. (1)", g.dt, lim);
  inside.assign((size_t)nx * ny, 0);
  const fdtd_pml& pm = p->pml;
  if (L.pml && (!std::isfinite(pm.m) || !std::isfinite(pm.sigma_scale) || pm.sigma_scale < 0 ||
                !std::isfinite(pm.kappa_max) || !std::isfinite(pm.alpha_max)))
    return fail(FDTD_EINVAL, "absorbing-layer parameters must be finite, sigma_scale >= 0");
  for (int k = 0; k < p->nroms && L.pml; ++k) {
    const fdtd_rom& r = p->roms[k];
    if (r.i0 - 1 < pm.n_xlo || r.i0 + r.ni > nx - 1 - pm.n_xhi || r.j0 - 1 < pm.n_ylo ||
        r.j0 + r.nj > ny - 1 - pm.n_yhi)
      return fail(FDTD_EINVAL, "region %d: it and its one-cell ring must lie outside the absorbing layers", k);
  }
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& r = p->roms[k];
    if (r.i0 < 1 || r.j0 < 1 || r.i0 + r.ni > nx - 1 || r.j0 + r.nj > ny - 1)
      return fail(FDTD_EINVAL, "region %d must keep one coarse cell to every wall", k);
  }
  for (int k = 0; k < p->nroms; ++k) {
    const fdtd_rom& a = p->roms[k];
    for (int m = 0; m < p->nroms; ++m) {
      if (m == k) continue;
      const fdtd_rom& b = p->roms[m];
      const bool sep = a.i0 + a.ni + 1 <= b.i0 || b.i0 + b.ni <= a.i0 - 1 ||
                       a.j0 + a.nj + 1 <= b.j0 || b.j0 + b.nj <= a.j0 - 1;
      if (!sep) return fail(FDTD_EINVAL, "regions %d and %d: one-cell rings overlap", k, m);
    }
    for (int j = a.j0; j < a.j0 + a.nj; ++j)
      for (int i = a.i0; i < a.i0 + a.ni; ++i) {
        if (g.pec && g.pec[(size_t)j * nx + i])
          return fail(FDTD_EINVAL, "region %d: PEC cell (%d,%d) inside the region (describe it in the model)", k, i, j);
        inside[(size_t)j * nx + i] = 1;
      }
    // a PEC ring cell pins the interface edge it shares with the region:
    // the model must leave that port undriven
    const int np = ports_of(a);
    for (int c = 0; c < np; ++c) {
      const PortCell pc = port_cell(a, c);
      if (!(g.pec && g.pec[(size_t)pc.oj * nx + pc.oi])) continue;
      for (int q = 0; q < a.q; ++q)
        if (a.Lt[(size_t)q * np + c] != 0.0)
          return fail(FDTD_EINVAL, "region %d: port %d faces PEC cell (%d,%d) but its column of Lt is not zero", k,
                      c, pc.oi, pc.oj);
    }
  }
  auto is_pec = [&](int i, int j) { return g.pec && g.pec[(size_t)j * nx + i]; };
  auto cell_ok = [&](int i, int j) {
    return i >= 0 && i < nx && j >= 0 && j < ny && !inside[(size_t)j * nx + i] && !is_pec(i, j);
  };
  auto active = [&](int comp, int i, int j) -> bool {
    if (comp == FDTD_HZ) return cell_ok(i, j);
    if (comp == FDTD_EX) return i >= 0 && i < nx && j >= 1 && j <= ny - 1 && cell_ok(i, j) && cell_ok(i, j - 1);
    if (comp == FDTD_EY) return j >= 0 && j < ny && i >= 1 && i <= nx - 1 && cell_ok(i, j) && cell_ok(i - 1, j);
    return false;
  };
  for (int k = 0; k < p->nsources; ++k) {
    const fdtd_source& s = p->sources[k];
    if (s.comp < 0 || s.comp > 2) return fail(FDTD_EINVAL, "source %d: bad component", k);
    if (!s.incr || s.nt < p->max_steps) return fail(FDTD_EINVAL, "source %d: needs max_steps increments", k);
    if (s.i0 >= s.i1 || s.j0 >= s.j1) return fail(FDTD_EINVAL, "source %d: empty rectangle", k);
    for (int j = s.j0; j < s.j1; ++j)
      for (int i = s.i0; i < s.i1; ++i)
        if (!active(s.comp, i, j))
          return fail(FDTD_EINVAL, "source %d: (%d,%d) is not updated by the coarse stencil", k, i, j);
  }
  for (int k = 0; k < p->nprobes; ++k) {
    const fdtd_probe& pr = p->probes[k];
    if (!active(pr.comp, pr.i, pr.j))
      return fail(FDTD_EINVAL, "probe %d: (%d,%d) comp %d is not a coarse-stencil sample", k, pr.i, pr.j, pr.comp);
  }
  // shared-matrix groups must really be identical
  for (int k = 0; k < p->nroms; ++k) {
    const int rep = L.slot_rep[L.slot_of_rom[k]];
    if (rep == k) continue;
    const fdtd_rom& a = p->roms[rep];
    const fdtd_rom& b = p->roms[k];
    const int q = a.q, np = ports_of(a);
    if (b.q != q || b.ni != a.ni || b.nj != a.nj)
      return fail(FDTD_EINVAL, "region %d: group %d members differ in shape", k, b.group);
    if ((a.Rt != b.Rt && std::memcmp(a.Rt, b.Rt, sizeof(double) * q * q)) ||
        (a.Ft != b.Ft && std::memcmp(a.Ft, b.Ft, sizeof(double) * q * q)) ||
        (a.Lt != b.Lt && std::memcmp(a.Lt, b.Lt, sizeof(double) * q * np)))
      return fail(FDTD_EINVAL, "region %d: group %d members have different matrices", k, b.group);
    // identical surroundings (interface half cells, PEC ring cells)
    auto ring = [&](const fdtd_rom& r, int c, double& e, double& s, bool& m) {
      const PortCell pc = port_cell(r, c);
      const size_t ci = (size_t)pc.oj * nx + pc.oi;
      e = g.eps_r ? g.eps_r[ci] : 1.0;
      s = g.sigma ? g.sigma[ci] : 0.0;
      m = g.pec && g.pec[ci];
    };
    for (int c = 0; c < np; ++c) {
      double e1, s1, e2, s2;
      bool m1, m2;
      ring(a, c, e1, s1, m1);
      ring(b, c, e2, s2, m2);
      if (e1 != e2 || s1 != s2 || m1 != m2)
        return fail(FDTD_EINVAL, "region %d: group %d members sit in different material", k, b.group);
    }
  }
  return FDTD_OK;
}

}  // namespace

// Default rows per stencil wave.  A wave streams its segment with two rows
// of loads in flight, so the grid needs a few waves per SIMD (1024 SIMDs)
// to hide memory latency: 16 rows while that still gives >= 4096 waves and
// the working set (~32 B per cell) stays cache-resident; otherwise 8 rows
// for large grids (HBM-bound, >= 8192 waves) and 4 for small ones.
int fdtd::default_tiling(int nx, int ny, int ts) {
  const long tx = (nx + kWave - 1) / kWave;
  auto waves = [&](int seg) { return tx * ((ny + seg - 1) / seg); };
  const double bytes = 4.0 * ts * (double)nx * (double)ny * 2.0;  // FP32: 32 B per cell
  if (waves(16) >= 4096 && bytes <= 192.0 * (1 << 20)) return 16;
  if (waves(8) >= 8192) return 8;
  return 4;
}

// Default rows per wave of the two-step launches (60 owned columns per
// wave): 16 while the launch still holds >= 4096 waves and the three field
// sets and the material stay Infinity-Cache resident (2048^2 FP32: 14.8 us
// per step at 16 rows, 15.0 at 8), else 4: more waves in flight beat the
// extra halo rows they read (8192^2: 243.8 us per step at 4 rows, 248.9 at
// 8, 268.7 at 16; 4096^2 with 256 copies of one model: 80.8, 82.1, 93.4).
int fdtd::default_tiling2(int nx, int ny, int ts) {
  const long tx = (nx + kOwned2 - 1) / kOwned2;
  auto waves = [&](int seg) { return tx * ((ny + seg - 1) / seg); };
  const double bytes = (9.0 * ts + 2.0) * (double)nx * (double)ny;  // three field sets + material index
  if (waves(16) >= 4096 && bytes <= 192.0 * (1 << 20)) return 16;
  return 4;
}

// a stencil workgroup covers 64 columns x (4 waves x seg rows)
void fdtd::set_tiling(fdtd_rom_sim* s, int seg) {
  s->seg = seg;
  const int rows = (kBlock / kWave) * seg;
  const int tx = (s->nx + kWave - 1) / kWave;
  const int nst = tx * ((s->ny + rows - 1) / rows);
  s->sp_f.nst_blocks = nst;
  s->sp_d.nst_blocks = nst;
  s->sp_f.tiles_x = tx;
  s->sp_d.tiles_x = tx;
  s->sp_f.seg = seg;
  s->sp_d.seg = seg;
}

// Tile roles of the two-step launches for the handle's tiling.  A tile of
// kOwned2 columns x 4 SEG rows is far when everything its two-step sweep
// reads (columns iw-2 .. iw+63, rows j0-2 .. j1+1, widened by one) stays
// clear of every region's zone [i0-2, i0+ni+1] x [j0-2, j0+nj+1] (the
// region, its ring of port cells and the edges between them, with one
// cell to spare) and of every source rectangle (widened by one); otherwise
// it is near.  Every cell whose step-(n+1) values the second launch's band
// blocks read (ring cells, their neighbours and the neighbours' edges) is
// owned by a near tile.  Uploaded synchronously (never while capturing).
template <typename T>
int fdtd::prepare_tb(fdtd_rom_sim* s) {
  const Layout& L = s->L;
  if (s->tb_seg == s->seg) return FDTD_OK;
  const int rows = (kBlock / kWave) * s->seg;
  const int tx2 = (s->nx + kOwned2 - 1) / kOwned2;
  const int nt = tx2 * ((s->ny + rows - 1) / rows);
  if (nt > L.max_tiles2) return fail(FDTD_EINVAL, "internal: two-step tile count %d exceeds %d", nt, L.max_tiles2);
  std::vector<uint8_t> role(nt, 0);
  std::vector<int> near;
  for (int t = 0; t < nt; ++t) {
    const int iw = (t % tx2) * kOwned2;
    const int jb0 = (t / tx2) * rows;
    const int jb1 = std::min(jb0 + rows, s->ny);
    const int fx0 = iw - 3, fx1 = iw + kWave, fy0 = jb0 - 3, fy1 = jb1 + 2;
    for (const RomHost& h : s->roms) {
      const int zx0 = h.i0 - 2, zx1 = h.i0 + h.ni + 1, zy0 = h.j0 - 2, zy1 = h.j0 + h.nj + 1;
      if (fx0 <= zx1 && zx0 <= fx1 && fy0 <= zy1 && zy0 <= fy1) role[t] = 1;
    }
    // the far-tile code holds no source terms
    const StepParams<T>& sp = step_params<T>(s);
    for (int k = 0; k < sp.nsrc; ++k) {
      const Src<T>& so = sp.src[k];
      if (fx0 <= so.i1 && so.i0 - 1 <= fx1 && fy0 <= so.j1 && so.j0 - 1 <= fy1) role[t] = 1;
    }
    if (role[t]) near.push_back(t);
  }
  hipStream_t st = s->stream;
  if (hipMemcpyAsync(s->ws + L.off_role2, role.data(), role.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      (!near.empty() && hipMemcpyAsync(s->ws + L.off_near, near.data(), near.size() * sizeof(int),
                                       hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(FDTD_EDEVICE, "two-step tile upload failed");
  // pieces of near tiles and the far tiles' share in the second launch
  // (set_pair_split; the default keeps every far tile in the first launch
  // where the whole grid's tiles are resident at once, else moves a share
  // that runs beside the second launch's coupling blocks)
  const int resident = 256 * 7;  // two-step tiles the GPU holds at once (256 CUs, 7 per CU)
  // the long chain of a shared model's MFMA GEMM blocks is worth hiding
  // under far tiles (4096^2 with 256 copies of one order-128 model: 176 ->
  // 155 us per pair at 50 % with 8-row waves; with 4-row waves per step
  // 82.5 us at 30 %, 79.4 at 40, 80.1 at 50, 77.8 at 60, 77.9 at 70);
  // row-parallel GEMV blocks are short (8192^2 with 256 models of orders
  // 32-96, 4-row waves: 243.3 us per step at 0 %, 252-260 at 5-30 %)
  bool gemm = false;
  for (size_t sl = 0; sl < L.slot_gemm.size(); ++sl) gemm = gemm || (L.slot_gemm[sl] && s->shared_gemm);
  const int split_pct = s->pair_split >= 0 ? s->pair_split : (nt > resident && gemm ? 60 : 0);
  const int near_rows = nt <= resident ? 2 : s->seg;
  auto fill = [&](auto& sp) {
    sp.tiles_x2 = tx2;
    sp.nst2_blocks = nt;
    sp.n_near = (int)near.size();
    sp.n_band = s->nroms;
    sp.near_rows = near_rows;
    sp.far_split = nt - (int)((int64_t)nt * split_pct / 100);
    sp.role2 = (const uint8_t*)(s->ws + L.off_role2);
    sp.near_list = (const int*)(s->ws + L.off_near);
    sp.st1m = (const uint8_t*)(s->ws + L.off_st1m);
  };
  fill(s->sp_f);
  fill(s->sp_d);
  s->tb_seg = s->seg;
  return FDTD_OK;
}

template int fdtd::prepare_tb<float>(fdtd_rom_sim*);
template int fdtd::prepare_tb<double>(fdtd_rom_sim*);

namespace {

int ev_pair(fdtd_rom_sim* s, std::vector<std::pair<hipEvent_t, hipEvent_t>>& pool, size_t& used,
            hipEvent_t& a, hipEvent_t& b) {
  if (used >= pool.size()) {
    hipEvent_t x, y;
    // timing-only events: no system-scope release/acquire (no cache flush
    // between the launches being timed)
    if (hipEventCreateWithFlags(&x, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&y, hipEventDisableSystemFence) != hipSuccess)
      return fail(FDTD_EDEVICE, "hipEventCreate failed");
    pool.emplace_back(x, y);
  }
  a = pool[used].first;
  b = pool[used].second;
  ++used;
  return FDTD_OK;
}

// Enqueue nsteps steps, the probe flush and the tick on `stream`, the
// handle's state standing at step steps0.  With two-step launches the steps
// go in pairs (a last odd step as a single launch); each pair leaves step
// n+2 in the set that held n+1's place, so the two sets trade places.
// Returns the number of pairs through `pairs`.
template <typename T>
int enqueue_steps(fdtd_rom_sim* s, int nsteps, hipStream_t stream, bool prof, int steps0, int* pairs,
                  bool allow_pairs = true) {
  StepParams<T> sp = step_params<T>(s);
  int k = 0;
  *pairs = 0;
  auto ev_begin = [&](hipEvent_t& e0, hipEvent_t& e1) -> int {
    const int rc = ev_pair(s, s->ev_st, s->used_st, e0, e1);
    if (rc != FDTD_OK) return rc;
    if (hipEventRecord(e0, stream) != hipSuccess) return fail(FDTD_EDEVICE, "hipEventRecord failed");
    return FDTD_OK;
  };
  if (s->tb && allow_pairs) {
    T* fc[3];
    for (int c = 0; c < 3; ++c) fc[c] = (T*)(s->ws + s->L.off_fc + c * s->L.field_elems * sizeof(T));
    for (; k + 2 <= nsteps; k += 2) {
      const int par = (steps0 + k) & 1;
      StepParams<T> a = sp, b = sp;
      for (int c = 0; c < 3; ++c) {
        a.f[par ^ 1][c] = fc[c];
        a.f2[c] = sp.f[par ^ 1][c];
        b.f[par ^ 1][c] = fc[c];
        b.f[par][c] = sp.f[par ^ 1][c];
        b.f2[c] = sp.f[par][c];  // the second launch's far tiles read step n
      }
      a.step_off = k;
      b.step_off = k + 1;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) {
        const int rc = ev_begin(e0, e1);
        if (rc != FDTD_OK) return rc;
      }
      if (launch_step2<T>(a, b, s->seg, s->smem, stream) != hipSuccess)
        return fail(FDTD_EDEVICE, "two-step launch failed: %s", hipGetErrorString(hipGetLastError()));
      if (prof && hipEventRecord(e1, stream) != hipSuccess) return fail(FDTD_EDEVICE, "hipEventRecord failed");
      for (int c = 0; c < 3; ++c) std::swap(sp.f[0][c], sp.f[1][c]);
      ++*pairs;
    }
  }
  for (; k < nsteps; ++k) {
    sp.step_off = k;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
      const int rc = ev_begin(e0, e1);
      if (rc != FDTD_OK) return rc;
    }
    if (launch_step<T>(sp, s->seg, s->smem, stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "step launch failed: %s", hipGetErrorString(hipGetLastError()));
    if (prof && hipEventRecord(e1, stream) != hipSuccess) return fail(FDTD_EDEVICE, "hipEventRecord failed");
  }
  // record the last probe row of the batch, then advance the device step base
  hipEvent_t e2 = nullptr, e3 = nullptr;
  if (prof) {
    const int rc = ev_pair(s, s->ev_cp, s->used_cp, e2, e3);
    if (rc != FDTD_OK) return rc;
    if (hipEventRecord(e2, stream) != hipSuccess) return fail(FDTD_EDEVICE, "hipEventRecord failed");
  }
  sp.step_off = nsteps;
  if (launch_probe_flush<T>(sp, stream) != hipSuccess || launch_tick(sp.ctrl, nsteps, stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "probe/tick launch failed");
  if (prof && hipEventRecord(e3, stream) != hipSuccess) return fail(FDTD_EDEVICE, "hipEventRecord failed");
  return FDTD_OK;
}

void drop_graph(fdtd_rom_sim* s) {
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  s->graph = nullptr;
  s->graph_steps = 0;
}

// Capture one batch of graph_batch steps (step kernels + flush + tick) on the
// library's own stream; it is replayed on the caller's stream.  Every launch
// reads its step index from the device base, so one graph serves any start.
template <typename T>
int capture_graph(fdtd_rom_sim* s, int gb, int key) {
  drop_graph(s);
  if (!s->cap_stream && hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamCreateWithFlags failed");
  if (hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamBeginCapture failed");
  int pairs = 0;
  int rc = enqueue_steps<T>(s, gb, s->cap_stream, false, s->steps, &pairs);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  if (rc == FDTD_OK && (pairs & 1)) rc = fail(FDTD_EINVAL, "internal: odd pair count in a captured batch");
  if (rc != FDTD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return fail(FDTD_EDEVICE, "hipStreamEndCapture failed");
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return fail(FDTD_EDEVICE, "hipGraphInstantiate failed");
  s->graph = ex;
  s->graph_steps = gb;
  s->graph_seg = s->seg;
  s->graph_key = key;
  return FDTD_OK;
}

// A captured batch holds fixed set pointers.  Single-step batches serve any
// start; two-step batches (a multiple of 4 steps: an even number of pairs,
// so the sets are back in place afterwards) are keyed on the start parity
// and the set order they were captured for.
int graph_key(const fdtd_rom_sim* s) { return s->tb ? 1 | ((s->steps & 1) << 1) | (s->flip << 2) : 0; }

int graph_batch_steps(const fdtd_rom_sim* s) { return s->tb ? s->graph_batch / 4 * 4 : s->graph_batch; }

template <typename T>
int ensure_graph(fdtd_rom_sim* s) {
  const int gb = graph_batch_steps(s);
  const int key = graph_key(s);
  if (!s->graph || s->graph_steps != gb || s->graph_seg != s->seg || s->graph_key != key)
    return capture_graph<T>(s, gb, key);
  return FDTD_OK;
}

// Launch the finiteness check on the physical field set holding the state
// after `at` steps (the handle's flip bit already current).
template <typename T>
int launch_check(fdtd_rom_sim* s, int at) {
  const Layout& L = s->L;
  const int set = (at & 1) ^ s->flip;
  const T* f = (const T*)(s->ws + L.off_fields + (size_t)3 * set * L.field_elems * sizeof(T));
  if (launch_finite_check<T>(f, 3 * L.field_elems, (int*)(s->ws + L.off_ctrl) + 2, s->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "finiteness check launch failed: %s", hipGetErrorString(hipGetLastError()));
  return FDTD_OK;
}

template <typename T>
int run_steps(fdtd_rom_sim* s, int nsteps) {
  if (nsteps == 0) return FDTD_OK;
  if (s->tb) {
    const int rc = prepare_tb<T>(s);
    if (rc != FDTD_OK) return rc;
  }
  int done = 0;
  bool checked = false;
  // after k more steps (state now at `at` steps): check every check_every
  auto after = [&](int k, int at) -> int {
    s->since_check += k;
    if (s->check_every > 0 && s->since_check >= s->check_every) {
      const int rc = launch_check<T>(s, at);
      if (rc != FDTD_OK) return rc;
      s->since_check = 0;
      checked = true;
    }
    return FDTD_OK;
  };
  const int gb = graph_batch_steps(s);
  if (gb > 0 && !s->prof && nsteps >= gb) {
    int rc = ensure_graph<T>(s);
    if (rc != FDTD_OK) return rc;
    while (nsteps - done >= gb) {
      if (hipGraphLaunch(s->graph, s->stream) != hipSuccess)
        return fail(FDTD_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(hipGetLastError()));
      done += gb;
      if ((rc = after(gb, s->steps + done)) != FDTD_OK) return rc;
    }
  }
  // direct launches, in chunks that end where a check is due (even-sized
  // where possible, so two-step runs keep their pairs)
  while (nsteps > done) {
    int c = nsteps - done;
    if (s->check_every > 0) {
      c = std::min(c, std::max(s->check_every - s->since_check, 1));
      if (s->tb && (c & 1) && c < nsteps - done) ++c;
    }
    int pairs = 0;
    int rc = enqueue_steps<T>(s, c, s->stream, s->prof, s->steps + done, &pairs);
    if (rc != FDTD_OK) return rc;
    if (pairs & 1) {
      StepParams<T>& sp = step_params<T>(s);
      for (int k = 0; k < 3; ++k) std::swap(sp.f[0][k], sp.f[1][k]);
      s->flip ^= 1;
    }
    done += c;
    if ((rc = after(c, s->steps + done)) != FDTD_OK) return rc;
  }
  s->steps += nsteps;
  if (checked) {
    int flag = 0;
    if (hipMemcpyAsync(&flag, (int*)(s->ws + s->L.off_ctrl) + 2, sizeof(int), hipMemcpyDeviceToHost,
                       s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "finiteness flag read failed: %s", hipGetErrorString(hipGetLastError()));
    if (flag)
      return fail(FDTD_EUNSTABLE, "non-finite field value found by the periodic check (state at step %d)",
                  s->steps);
  }
  return FDTD_OK;
}

template <typename T>
int prepare_run(fdtd_rom_sim* s, int nsteps) {
  if (s->tb) {
    const int rc = prepare_tb<T>(s);
    if (rc != FDTD_OK) return rc;
  }
  const int gb = graph_batch_steps(s);
  if (gb > 0 && !s->prof && nsteps >= gb) return ensure_graph<T>(s);
  return FDTD_OK;
}

template <typename T>
void to_double(const std::vector<char>& raw, size_t n, double* out) {
  const T* t = (const T*)raw.data();
  for (size_t k = 0; k < n; ++k) out[k] = (double)t[k];
}

// nsteps single-step launches (no pairs, no graph, no finiteness check, no
// host allocation), then the probe flush and the tick.
template <typename T>
int run_direct(fdtd_rom_sim* s, int nsteps) {
  if (nsteps == 0) return FDTD_OK;
  int pairs = 0;
  const int rc = enqueue_steps<T>(s, nsteps, s->stream, false, s->steps, &pairs, false);
  if (rc != FDTD_OK) return rc;
  s->steps += nsteps;
  return FDTD_OK;
}

}  // namespace

int fdtd::run_steps_any(fdtd_rom_sim* s, int nsteps) {
  return s->dtype == FDTD_F32 ? run_steps<float>(s, nsteps) : run_steps<double>(s, nsteps);
}

int fdtd::run_direct_any(fdtd_rom_sim* s, int nsteps) {
  return s->dtype == FDTD_F32 ? run_direct<float>(s, nsteps) : run_direct<double>(s, nsteps);
}

extern "C" {

const char* fdtd_rom_strerror(int status) {
  switch (status) {
    case FDTD_OK: return "ok";
    case FDTD_EINVAL: return "invalid argument";
    case FDTD_ENOMEM: return "out of memory / workspace too small";
    case FDTD_EDEVICE: return "HIP device error";
    case FDTD_ENOTPASSIVE: return "reduced model not passive at this time step";
    case FDTD_EUNSTABLE: return "non-finite field (instability)";
    case FDTD_ESTATE: return "invalid state for this call";
    default: return "unknown status";
  }
}

const char* fdtd_rom_last_error(void) { return g_err.c_str(); }

int fdtd_rom_workspace_size(const fdtd_problem* prob, size_t* bytes) {
  if (!bytes) return fail(FDTD_EINVAL, "null output");
  try {
    Layout L;
    const int rc = plan_problem(prob, L);
    if (rc != FDTD_OK) return rc;
    *bytes = L.total;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_create(const fdtd_problem* prob, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                    fdtd_rom_sim** out) {
  if (!out) return fail(FDTD_EINVAL, "null output handle");
  *out = nullptr;
  try {
    Layout L;
    int rc = plan_problem(prob, L);
    if (rc != FDTD_OK) return rc;
    if (!dev_workspace) return fail(FDTD_EINVAL, "null workspace");
    if (((uintptr_t)dev_workspace) % 256) return fail(FDTD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(FDTD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    std::vector<unsigned char> inside;
    rc = validate_numbers(prob, L, inside);
    if (rc != FDTD_OK) return rc;
    fdtd_rom_sim* s = new fdtd_rom_sim();
    s->dtype = prob->grid.dtype;
    s->nx = prob->grid.nx;
    s->ny = prob->grid.ny;
    s->pitch = L.pitch;
    s->dx = prob->grid.dx;
    s->dy = prob->grid.dy;
    s->dt = prob->grid.dt;
    s->max_steps = prob->max_steps;
    s->nprobes = prob->nprobes;
    s->nsrc = prob->nsources;
    s->nroms = prob->nroms;
    if (prob->nprobes > 0) s->probes.assign(prob->probes, prob->probes + prob->nprobes);
    if (prob->grid.pec)
      for (size_t c = 0; c < (size_t)s->nx * s->ny; ++c)
        if (prob->grid.pec[c]) {
          s->pec.assign(prob->grid.pec, prob->grid.pec + (size_t)s->nx * s->ny);
          break;
        }
    s->stream = (hipStream_t)hip_stream;
    s->ws = (char*)dev_workspace;
    s->L = L;
    rc = coupling_precompute(prob, s->roms);
    if (rc == FDTD_OK)
      rc = (s->dtype == FDTD_F32) ? setup_device<float>(s, prob, inside)
                                  : setup_device<double>(s, prob, inside);
    s->tb = L.tb_ok;  // two steps per pass wherever the grid allows it
    if (rc == FDTD_OK)
      set_tiling(s, s->tb ? default_tiling2(s->nx, s->ny, (int)L.tsize) : default_tiling(s->nx, s->ny, (int)L.tsize));
    if (rc != FDTD_OK) {
      delete s;
      return rc;
    }
    *out = s;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_step(fdtd_rom_sim* sim) { return fdtd_rom_run(sim, 1); }

int fdtd_rom_run(fdtd_rom_sim* sim, int32_t nsteps) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (nsteps < 0) return fail(FDTD_EINVAL, "negative step count");
  if ((int64_t)sim->steps + nsteps > sim->max_steps)
    return fail(FDTD_ESTATE, "%d + %d steps exceed max_steps=%d", sim->steps, nsteps, sim->max_steps);
  return run_steps_any(sim, nsteps);
}

int fdtd_rom_prepare_run(fdtd_rom_sim* sim, int32_t nsteps) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (nsteps < 0) return fail(FDTD_EINVAL, "negative step count");
  return sim->dtype == FDTD_F32 ? prepare_run<float>(sim, nsteps) : prepare_run<double>(sim, nsteps);
}

int fdtd_rom_set_check_interval(fdtd_rom_sim* sim, int32_t every) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (every < 0) return fail(FDTD_EINVAL, "check interval must be >= 0");
  sim->check_every = every;
  sim->since_check = 0;
  return FDTD_OK;
}

int fdtd_rom_get_check_interval(const fdtd_rom_sim* sim, int32_t* every) {
  if (!sim || !every) return fail(FDTD_EINVAL, "null argument");
  *every = sim->check_every;
  return FDTD_OK;
}

int fdtd_rom_steps_done(const fdtd_rom_sim* sim, int32_t* n) {
  if (!sim || !n) return fail(FDTD_EINVAL, "null argument");
  *n = sim->steps;
  return FDTD_OK;
}

int fdtd_rom_read_probes(const fdtd_rom_sim* sim, int32_t first, int32_t count, double* host_out) {
  if (!sim || (!host_out && count > 0)) return fail(FDTD_EINVAL, "null argument");
  if (first < 0 || count < 0 || (int64_t)first + count > sim->steps)
    return fail(FDTD_EINVAL, "probe rows [%d, %d) outside the %d steps taken", first, first + count, sim->steps);
  const size_t n = (size_t)count * sim->nprobes;
  if (n == 0) return FDTD_OK;
  const size_t ts = sim->L.tsize;
  std::vector<char> raw(n * ts);
  if (hipMemcpyAsync(raw.data(), sim->ws + sim->L.off_pbuf + (size_t)first * sim->nprobes * ts, n * ts,
                     hipMemcpyDeviceToHost, sim->stream) != hipSuccess ||
      hipStreamSynchronize(sim->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "probe read failed: %s", hipGetErrorString(hipGetLastError()));
  if (ts == 4) to_double<float>(raw, n, host_out);
  else to_double<double>(raw, n, host_out);
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(host_out[k])) return fail(FDTD_EUNSTABLE, "non-finite probe value at row %zu", first + k / sim->nprobes);
  return FDTD_OK;
}

int fdtd_rom_probe_objective(const fdtd_rom_sim* sim, int32_t probe, int32_t first, int32_t count, double* J) {
  if (!sim || !J) return fail(FDTD_EINVAL, "null argument");
  if (probe < 0 || probe >= sim->nprobes || sim->probes[probe].comp != FDTD_HZ)
    return fail(FDTD_EINVAL, "probe %d is not an Hz probe of this problem", probe);
  std::vector<double> pr((size_t)count * sim->nprobes);
  const int rc = fdtd_rom_read_probes(sim, first, count, pr.data());
  if (rc != FDTD_OK) return rc;
  double acc = 0;
  for (int n = 0; n < count; ++n) {
    const double v = pr[(size_t)n * sim->nprobes + probe];
    acc += v * v;
  }
  *J = sim->dt * acc;
  return FDTD_OK;
}

int fdtd_rom_read_field(const fdtd_rom_sim* sim, int32_t comp, double* host_out) {
  if (!sim || !host_out) return fail(FDTD_EINVAL, "null argument");
  if (comp < 0 || comp > 2) return fail(FDTD_EINVAL, "bad component");
  const size_t ts = sim->L.tsize, fe = sim->L.field_elems;
  std::vector<char> raw(fe * ts);
  const char* src = sim->ws + sim->L.off_fields + (3 * cur_set(sim) + comp) * fe * ts;
  if (hipMemcpyAsync(raw.data(), src, fe * ts, hipMemcpyDeviceToHost, sim->stream) != hipSuccess ||
      hipStreamSynchronize(sim->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "field read failed");
  std::vector<double> d(fe);
  if (ts == 4) to_double<float>(raw, fe, d.data());
  else to_double<double>(raw, fe, d.data());
  const int nx = sim->nx, ny = sim->ny, P = sim->pitch;
  if (comp == FDTD_HZ) {
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) host_out[(size_t)j * nx + i] = d[(size_t)j * P + i];
  } else if (comp == FDTD_EX) {
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) host_out[(size_t)j * nx + i] = j < ny ? d[(size_t)j * P + i] : 0.0;
  } else {
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i <= nx; ++i) host_out[(size_t)j * (nx + 1) + i] = i < nx ? d[(size_t)j * P + i] : 0.0;
  }
  return FDTD_OK;
}

int fdtd_rom_read_rom_state(const fdtd_rom_sim* sim, int32_t k, double* host_out) {
  if (!sim || !host_out) return fail(FDTD_EINVAL, "null argument");
  if (k < 0 || k >= sim->nroms) return fail(FDTD_EINVAL, "region index out of range");
  const size_t ts = sim->L.tsize;
  const int q = sim->roms[k].q;
  std::vector<char> raw((size_t)q * ts);
  // x~^n sits in the buffer of parity n (eq. (23) writes the other one)
  const size_t xo = sim->L.x_off[k] + (size_t)(sim->steps & 1) * (((size_t)q + 63) / 64 * 64);
  if (hipMemcpyAsync(raw.data(), sim->ws + sim->L.off_xs + xo * ts, q * ts, hipMemcpyDeviceToHost,
                     sim->stream) != hipSuccess ||
      hipStreamSynchronize(sim->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "state read failed");
  if (ts == 4) to_double<float>(raw, q, host_out);
  else to_double<double>(raw, q, host_out);
  return FDTD_OK;
}

int fdtd_rom_coupled_update(const fdtd_problem* prob, int32_t k, double* A, double* B, double* C) {
  try {
    Layout L;
    int rc = plan_problem(prob, L);
    if (rc != FDTD_OK) return rc;
    if (k < 0 || k >= prob->nroms) return fail(FDTD_EINVAL, "region index out of range");
    std::vector<unsigned char> inside;
    rc = validate_numbers(prob, L, inside);
    if (rc != FDTD_OK) return rc;
    std::vector<RomHost> roms;
    rc = coupling_precompute(prob, roms);
    if (rc != FDTD_OK) return rc;
    const RomHost& h = roms[k];
    if (A) std::memcpy(A, h.A.data(), h.A.size() * sizeof(double));
    if (B) std::memcpy(B, h.B.data(), h.B.size() * sizeof(double));
    if (C) std::memcpy(C, h.C.data(), h.C.size() * sizeof(double));
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_energy(const fdtd_rom_sim* sim, double* e) {
  if (!sim || !e) return fail(FDTD_EINVAL, "null argument");
  try {
    const Layout& L = sim->L;
    const size_t ts = L.tsize, fe = L.field_elems;
    const char* set = sim->ws + L.off_fields + (size_t)cur_set(sim) * 3 * fe * ts;
    double* part = (double*)(sim->ws + L.off_energy);
    const double ch = kMu0 * sim->dx * sim->dy / sim->dt;
    const double ha = 0.5 * sim->dx * sim->dy;
    hipError_t err;
    if (ts == 4)
      err = launch_energy<float>((const float*)set, (const float*)set + fe, (const float*)set + 2 * fe,
                                 (const float*)(sim->ws + L.off_al), sim->nx, sim->ny, sim->pitch, ch, ha,
                                 sim->dx, sim->dy, part, sim->stream);
    else
      err = launch_energy<double>((const double*)set, (const double*)set + fe, (const double*)set + 2 * fe,
                                  (const double*)(sim->ws + L.off_al), sim->nx, sim->ny, sim->pitch, ch, ha,
                                  sim->dx, sim->dy, part, sim->stream);
    if (err != hipSuccess) return fail(FDTD_EDEVICE, "energy launch failed: %s", hipGetErrorString(err));
    const int nb = energy_blocks(sim->nx, sim->ny);
    std::vector<double> h(nb);
    if (hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, sim->stream) != hipSuccess ||
        hipStreamSynchronize(sim->stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "energy read failed");
    double tot = 0;
    for (double v : h) tot += v;
    // reduced models: x~^T R~ x~
    for (int k = 0; k < sim->nroms; ++k) {
      const RomHost& r = sim->roms[k];
      std::vector<double> x(r.q);
      const int rc = fdtd_rom_read_rom_state(sim, k, x.data());
      if (rc != FDTD_OK) return rc;
      for (int a = 0; a < r.q; ++a) {
        double row = 0;
        for (int b = 0; b < r.q; ++b) row += r.R[(size_t)a * r.q + b] * x[b];
        tot += x[a] * row;
      }
    }
    *e = tot;
    if (!std::isfinite(tot)) return fail(FDTD_EUNSTABLE, "non-finite energy");
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

namespace {
constexpr int32_t kStateMagic = 0x46445453;  // state blob tag
constexpr size_t kStateHeader = 256;
struct StateHeader {
  int32_t magic, dtype, steps, nx, ny, pitch;
  int64_t field_elems, xs_elems;
  int32_t pml, pad;
};
// blob: header | current field set | reduced states | (layers) the two
// Hz auxiliary fields of the current parity, then those at Ex and Ey
size_t state_psi_off(const fdtd_rom_sim* s) {
  return kStateHeader + align_up(3 * s->L.field_elems * s->L.tsize, 256) +
         align_up(s->L.xs_elems * s->L.tsize, 256);
}
size_t state_bytes(const fdtd_rom_sim* s) {
  return state_psi_off(s) + (s->L.pml ? 4 * s->L.field_elems * s->L.tsize : 0);
}
// device address of auxiliary field k (0,1: Hz at parity par; 2,3: Ex, Ey)
char* psi_addr(const fdtd_rom_sim* s, int k, int par) {
  const size_t fb = s->L.field_elems * s->L.tsize;
  char* base = s->ws + s->L.off_psi;
  return k < 2 ? base + (size_t)(2 * par + k) * fb : base + (size_t)(2 + k) * fb;
}
}  // namespace

int fdtd_rom_state_size(const fdtd_rom_sim* sim, size_t* bytes) {
  if (!sim || !bytes) return fail(FDTD_EINVAL, "null argument");
  *bytes = state_bytes(sim);
  return FDTD_OK;
}

int fdtd_rom_get_state(const fdtd_rom_sim* sim, void* dev_dst) {
  if (!sim || !dev_dst) return fail(FDTD_EINVAL, "null argument");
  const Layout& L = sim->L;
  const size_t set_bytes = 3 * L.field_elems * L.tsize;
  StateHeader h{kStateMagic, sim->dtype, sim->steps, sim->nx, sim->ny, sim->pitch, (int64_t)L.field_elems,
                (int64_t)L.xs_elems, L.pml ? 1 : 0, 0};
  char* d = (char*)dev_dst;
  if (hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, sim->stream) != hipSuccess ||
      hipMemcpyAsync(d + kStateHeader, sim->ws + L.off_fields + (size_t)cur_set(sim) * set_bytes, set_bytes,
                     hipMemcpyDeviceToDevice, sim->stream) != hipSuccess ||
      (L.xs_elems > 0 && hipMemcpyAsync(d + kStateHeader + align_up(set_bytes, 256), sim->ws + L.off_xs,
                                        L.xs_elems * L.tsize, hipMemcpyDeviceToDevice, sim->stream) != hipSuccess))
    return fail(FDTD_EDEVICE, "state copy failed");
  const size_t fb = L.field_elems * L.tsize;
  for (int k = 0; k < 4 && L.pml; ++k)
    if (hipMemcpyAsync(d + state_psi_off(sim) + k * fb, psi_addr(sim, k, sim->steps & 1), fb,
                       hipMemcpyDeviceToDevice, sim->stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "state copy failed");
  if (hipStreamSynchronize(sim->stream) != hipSuccess) return fail(FDTD_EDEVICE, "state copy failed");
  return FDTD_OK;
}

int fdtd_rom_set_state(fdtd_rom_sim* sim, const void* dev_src) {
  if (!sim || !dev_src) return fail(FDTD_EINVAL, "null argument");
  const Layout& L = sim->L;
  const size_t set_bytes = 3 * L.field_elems * L.tsize;
  StateHeader h{};
  const char* d = (const char*)dev_src;
  if (hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, sim->stream) != hipSuccess ||
      hipStreamSynchronize(sim->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "state header read failed");
  if (h.magic != kStateMagic || h.dtype != sim->dtype || h.nx != sim->nx || h.ny != sim->ny ||
      h.pitch != sim->pitch || h.field_elems != (int64_t)L.field_elems || h.xs_elems != (int64_t)L.xs_elems ||
      h.pml != (L.pml ? 1 : 0))
    return fail(FDTD_EINVAL, "state blob does not belong to a handle of this problem shape");
  if (h.steps < 0 || h.steps > sim->max_steps)
    return fail(FDTD_EINVAL, "state at step %d outside [0, max_steps=%d]", h.steps, sim->max_steps);
  int ctrl[kCtrlInts] = {h.steps, 0, 0, 0};
  if (hipMemcpyAsync(sim->ws + L.off_fields + (size_t)((h.steps & 1) ^ sim->flip) * set_bytes, d + kStateHeader, set_bytes,
                     hipMemcpyDeviceToDevice, sim->stream) != hipSuccess ||
      (L.xs_elems > 0 && hipMemcpyAsync(sim->ws + L.off_xs, d + kStateHeader + align_up(set_bytes, 256),
                                        L.xs_elems * L.tsize, hipMemcpyDeviceToDevice, sim->stream) != hipSuccess) ||
      hipMemcpyAsync(sim->ws + L.off_ctrl, ctrl, sizeof(ctrl), hipMemcpyHostToDevice, sim->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "state copy failed");
  const size_t fb = L.field_elems * L.tsize;
  for (int k = 0; k < 4 && L.pml; ++k)
    if (hipMemcpyAsync(psi_addr(sim, k, h.steps & 1), d + state_psi_off(sim) + k * fb, fb,
                       hipMemcpyDeviceToDevice, sim->stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "state copy failed");
  if (hipStreamSynchronize(sim->stream) != hipSuccess) return fail(FDTD_EDEVICE, "state copy failed");
  sim->steps = h.steps;
  sim->since_check = 0;  // the control block copy above cleared the non-finite flag
  return FDTD_OK;
}

int fdtd_rom_profile_enable(fdtd_rom_sim* sim, int32_t enable) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  sim->prof = enable != 0;
  return FDTD_OK;
}

int fdtd_rom_profile_read(fdtd_rom_sim* sim, double* step_ms, int64_t* step_launches, double* tail_ms,
                          int64_t* tail_launches) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (hipStreamSynchronize(sim->stream) != hipSuccess) return fail(FDTD_EDEVICE, "synchronize failed");
  double a = 0, b = 0;
  for (size_t k = 0; k < sim->used_st; ++k) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, sim->ev_st[k].first, sim->ev_st[k].second) != hipSuccess)
      return fail(FDTD_EDEVICE, "hipEventElapsedTime failed");
    a += ms;
  }
  for (size_t k = 0; k < sim->used_cp; ++k) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, sim->ev_cp[k].first, sim->ev_cp[k].second) != hipSuccess)
      return fail(FDTD_EDEVICE, "hipEventElapsedTime failed");
    b += ms;
  }
  if (step_ms) *step_ms = a;
  if (step_launches) *step_launches = (int64_t)sim->used_st;
  if (tail_ms) *tail_ms = b;
  if (tail_launches) *tail_launches = (int64_t)sim->used_cp;
  sim->used_st = sim->used_cp = 0;
  return FDTD_OK;
}

int fdtd_rom_set_tiling(fdtd_rom_sim* sim, int32_t seg) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (seg != 4 && seg != 8 && seg != 16 && seg != 32) return fail(FDTD_EINVAL, "segment rows must be 4, 8, 16 or 32");
  set_tiling(sim, seg);
  return FDTD_OK;
}

int fdtd_rom_set_pair_split(fdtd_rom_sim* sim, int32_t percent) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (percent != -1 && (percent < 0 || percent > 90)) return fail(FDTD_EINVAL, "split must be -1 or 0..90 percent");
  sim->pair_split = percent;
  sim->tb_seg = 0;  // tile roles and launch shapes are rebuilt before the next pair
  drop_graph(sim);
  return FDTD_OK;
}

int fdtd_rom_get_pair_split(const fdtd_rom_sim* sim, int32_t* percent) {
  if (!sim || !percent) return fail(FDTD_EINVAL, "null argument");
  const StepParams<float>& sp = sim->sp_f;
  const StepParams<double>& sd = sim->sp_d;
  const int nt = sim->dtype == FDTD_F32 ? sp.nst2_blocks : sd.nst2_blocks;
  const int split = sim->dtype == FDTD_F32 ? sp.far_split : sd.far_split;
  *percent = (sim->tb_seg == sim->seg && nt > 0) ? (int)((int64_t)(nt - split) * 100 / nt) : sim->pair_split;
  return FDTD_OK;
}

int fdtd_rom_get_tiling(const fdtd_rom_sim* sim, int32_t* seg) {
  if (!sim || !seg) return fail(FDTD_EINVAL, "null argument");
  *seg = sim->seg;
  return FDTD_OK;
}

int fdtd_rom_set_shared_gemm(fdtd_rom_sim* sim, int32_t enable) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  const Layout& L = sim->L;
  const bool on = enable != 0;
  const RowBlock* b = (const RowBlock*)(sim->ws + (on ? L.off_blocks_mixed : L.off_blocks));
  const int nb = on ? L.nblocks_mixed : L.nrowblocks;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0) {
      sim->sp_f.blocks = b;
      sim->sp_f.nrowblocks = nb;
      sim->sp_f.ncoup_blocks = (nb + 7) / 8 * 8;
    } else {
      sim->sp_d.blocks = b;
      sim->sp_d.nrowblocks = nb;
      sim->sp_d.ncoup_blocks = (nb + 7) / 8 * 8;
    }
  }
  sim->smem = on ? L.smem_mixed : L.smem_gemv;
  sim->shared_gemm = on;
  sim->tb_seg = 0;  // the default far-tile split follows the coupling path
  drop_graph(sim);
  return FDTD_OK;
}

int fdtd_rom_set_material_mode(fdtd_rom_sim* sim, int32_t mode) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (mode != 0 && mode != 1) return fail(FDTD_EINVAL, "material mode must be 0 or 1");
  if (mode == 1 && sim->nmat == 0)
    return fail(FDTD_EINVAL, "material table unavailable: more than %d distinct (eps_r, sigma) pairs", kMaxMaterials);
  sim->sp_f.midx = mode;
  sim->sp_d.midx = mode;
  drop_graph(sim);
  return FDTD_OK;
}

int fdtd_rom_get_material_mode(fdtd_rom_sim* sim, int32_t* mode, int32_t* entries) {
  if (!sim || !mode || !entries) return fail(FDTD_EINVAL, "null argument");
  *mode = sim->dtype == FDTD_F32 ? sim->sp_f.midx : sim->sp_d.midx;
  *entries = sim->nmat;
  return FDTD_OK;
}

int fdtd_rom_set_time_blocking(fdtd_rom_sim* sim, int32_t on) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (on != 0 && on != 1) return fail(FDTD_EINVAL, "time blocking must be 0 or 1");
  if (on && !sim->L.tb_ok) return fail(FDTD_EINVAL, "two-step launches need a grid without absorbing layers");
  if (hipStreamSynchronize(sim->stream) != hipSuccess) return fail(FDTD_EDEVICE, "synchronize failed");
  sim->tb = on != 0;
  drop_graph(sim);
  return FDTD_OK;
}

int fdtd_rom_get_time_blocking(const fdtd_rom_sim* sim, int32_t* on) {
  if (!sim || !on) return fail(FDTD_EINVAL, "null argument");
  *on = sim->tb ? 1 : 0;
  return FDTD_OK;
}

int fdtd_rom_set_graph(fdtd_rom_sim* sim, int32_t batch) {
  if (!sim) return fail(FDTD_EINVAL, "null handle");
  if (batch < 0 || batch > 4096) return fail(FDTD_EINVAL, "graph batch must be in [0, 4096]");
  sim->graph_batch = batch;
  if (batch == 0) drop_graph(sim);
  return FDTD_OK;
}

void fdtd_rom_destroy(fdtd_rom_sim* sim) {
  if (!sim) return;
  (void)hipStreamSynchronize(sim->stream);
  drop_graph(sim);
  if (sim->cap_stream) (void)hipStreamDestroy(sim->cap_stream);
  for (auto& e : sim->ev_st) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : sim->ev_cp) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete sim;
}

}  // extern "C"
