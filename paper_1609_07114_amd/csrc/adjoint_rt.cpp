// Host orchestration of the reverse sweep (fdtd_rom_adjoint,
// fdtd_rom_adjoint_models, fdtd_rom_adjoint_noalloc).
//
// Forward: the handle runs nsteps as usual; before every segment of
// ckpt_every steps its current field set and reduced states are copied to a
// checkpoint.  Reverse, one segment at a time from the last: the segment's
// forward states are recomputed from its checkpoint with the step kernel
// writing each step's output into its own slot and its reduced states into
// its own image (nothing overwritten, no probe record, a private step
// counter), then the adjoint steps run from the segment's end back to its
// start, each reading E^n (slot n) and Hz^{n+1/2} (slot n+1).  A reverse
// step is one launch (the stream of step n beside eq. (23)'s transpose of
// step n-1); the sweep through the models keeps two launches per step, the
// transpose accumulating dJ/dG with x~^n of the segment's images.  Peak
// memory: checkpoints + one segment.
//
// Absorbing layers add the auxiliary fields: a checkpoint also holds the
// four of its step, a slot also the two at Ex and Ey (the reverse step
// weighs the stretched Hz differences with them), the recompute runs the
// two at Hz through a private ping-pong pair, and the adjoint sets carry
// the four adjoint auxiliary fields.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdtd_rom.h"
#include "adjoint.hpp"
#include "linalg.hpp"
#include "runtime.hpp"

using namespace fdtd;

namespace {

// Plain fields only: the layout is planned without allocating (the
// no-allocation entry point plans it too).
struct AdjLayout {
  int K = 0, nck = 0;
  // buffer sets of recomputed slots and images: 2 when the recompute of
  // the segment below runs on a second stream beside the reverse steps of
  // this one (at least two segments, not the no-allocation entry), else 1
  int nbuf = 1;
  size_t slots_stride = 0, xrec_stride = 0;  // bytes per buffer set
  size_t set_bytes = 0, xs_bytes = 0;
  size_t slot_bytes = 0, lam_bytes = 0, ck_psi = 0;  // per slot / adjoint set; checkpoint's psi offset
  size_t off_ctrl = 0, off_ckpt = 0, ck_stride = 0, off_slots = 0, off_xrec = 0, off_psih = 0;
  size_t off_lam = 0, off_lx = 0, off_g = 0, off_gseg = 0, off_gt = 0, off_roms = 0, off_j = 0;
  size_t off_rtab = 0, off_dgoff = 0, off_dg = 0, off_pend = 0, pend_bytes = 0, total = 0;
  size_t gt_elems = 0;
  size_t img = 0;        // elements per image of reduced states (one per step of a segment)
  bool models = false;   // gradients through the models: dJ/dG accumulators
  size_t dg_elems = 0;
};

// Element offset of region k's dJ/dG^T accumulator (ldg x ldg, regions in order).
size_t region_dg(const fdtd_rom_sim* s, int k) {
  size_t o = 0;
  for (int a = 0; a < k; ++a) {
    const size_t ldg = align_up((size_t)s->roms[a].q + s->roms[a].np, kWave);
    o += ldg * ldg;
  }
  return o;
}

// Element offset of matrix slot sl's G^T block (ldg x ldg, slots in order).
size_t slot_gt(const fdtd_rom_sim* s, size_t sl) {
  size_t ge = 0;
  for (size_t k = 0; k < sl; ++k) {
    const RomHost& h = s->roms[s->L.slot_rep[k]];
    const size_t ldg = align_up((size_t)h.q + h.np, kWave);
    ge = align_up(ge + ldg * ldg, 64);
  }
  return ge;
}

int plan_adjoint(const fdtd_rom_sim* s, int nsteps, int ckpt_every, AdjLayout& A, bool models = false,
                 bool pipelined = true) {
  if (nsteps < 1 || nsteps > s->max_steps)
    return fail(FDTD_EINVAL, "nsteps=%d outside [1, max_steps=%d]", nsteps, s->max_steps);
  if (ckpt_every < 0 || ckpt_every > nsteps)
    return fail(FDTD_EINVAL, "ckpt_every=%d outside [0, nsteps=%d]", ckpt_every, nsteps);
  const Layout& L = s->L;
  A.K = ckpt_every > 0 ? ckpt_every : (int)std::ceil(std::sqrt((double)nsteps));
  A.nck = (nsteps + A.K - 1) / A.K;
  A.nbuf = pipelined && A.nck >= 2 ? 2 : 1;
  const size_t ts = L.tsize;
  const size_t fb = L.field_elems * ts;
  A.set_bytes = 3 * fb;
  A.slot_bytes = (L.pml ? 5 : 3) * fb;   // Hz, Ex, Ey (+ psi at Ex, Ey)
  A.lam_bytes = (L.pml ? 7 : 3) * fb;    // + adjoints of the four psi
  A.xs_bytes = align_up(std::max<size_t>(L.xs_elems, 1) * ts, 256);
  A.gt_elems = slot_gt(s, L.slot_rep.size());
  size_t o = 0;
  A.off_ctrl = o;
  o = align_up(o + kCtrlInts * sizeof(int), 256);
  A.off_ckpt = o;
  A.ck_psi = align_up(A.set_bytes, 256) + A.xs_bytes;
  A.ck_stride = A.ck_psi + (L.pml ? align_up(4 * fb, 256) : 0);
  o += (size_t)A.nck * A.ck_stride;
  A.off_slots = o;
  A.slots_stride = align_up((size_t)A.K * A.slot_bytes, 256);
  o += A.nbuf * A.slots_stride;
  // reduced states of every step of a segment: K + 1 images (256-B aligned)
  A.img = align_up(std::max<size_t>(L.xs_elems, 1), 64);
  A.off_xrec = o;
  A.xrec_stride = align_up((size_t)(A.K + 1) * A.img * ts, 256);
  o += A.nbuf * A.xrec_stride;
  A.off_psih = o;
  o = align_up(o + (L.pml ? 4 * fb : 0), 256);
  A.off_lam = o;
  o = align_up(o + 2 * A.lam_bytes, 256);
  A.off_lx = o;
  o = align_up(o + 2 * A.xs_bytes, 256);
  // fused reverse steps (all but the sweep through the models): lambda_h of
  // eq. (23)'s transpose per ring cell, two field-shaped arrays (ping-pong)
  A.off_pend = o;
  A.pend_bytes = models ? 0 : 2 * fb;
  o = align_up(o + A.pend_bytes, 256);
  A.off_g = o;
  o = align_up(o + 2 * L.field_elems * sizeof(double), 256);
  A.off_gseg = o;  // FP32 runs: per-segment accumulators in FP32
  o = align_up(o + (ts == 4 ? 2 * L.field_elems * ts : 0), 256);
  A.off_gt = o;
  o = align_up(o + A.gt_elems * ts, 256);
  A.off_roms = o;
  o = align_up(o + (size_t)std::max(s->nroms, 1) * sizeof(RomDev), 256);
  A.off_j = o;  // the objective, when summed on the device
  o = align_up(o + sizeof(double), 256);
  A.off_rtab = o;  // the recompute's two model tables (xstride +img, -img)
  o = align_up(o + 2 * (size_t)std::max(s->nroms, 1) * sizeof(RomDev), 256);
  A.models = models;
  A.dg_elems = models ? region_dg(s, s->nroms) : 0;
  A.off_dgoff = o;  // models: per region the offset of its dJ/dG^T accumulator
  o = align_up(o + (models ? (size_t)std::max(s->nroms, 1) * sizeof(int64_t) : 0), 256);
  A.off_dg = o;
  o = align_up(o + A.dg_elems * sizeof(double), 256);
  A.total = o;
  // every part in order, disjoint, inside the total: the checkpoints (each
  // a field set, the reduced states and, with layers, four auxiliary
  // fields), the recompute slots, the scratch states, the recompute's psi
  // at Hz, the adjoint sets, adjoint states, accumulators, G^T, model table
  const size_t parts[][2] = {
      {A.off_ctrl, kCtrlInts * sizeof(int)},
      {A.off_ckpt, (size_t)A.nck * A.ck_stride},
      {A.off_slots, A.nbuf * A.slots_stride},
      {A.off_xrec, A.nbuf * A.xrec_stride},
      {A.off_psih, L.pml ? 4 * fb : 0},
      {A.off_lam, 2 * A.lam_bytes},
      {A.off_lx, 2 * A.xs_bytes},
      {A.off_pend, A.pend_bytes},
      {A.off_g, 2 * L.field_elems * sizeof(double)},
      {A.off_gseg, ts == 4 ? 2 * L.field_elems * ts : 0},
      {A.off_gt, A.gt_elems * ts},
      {A.off_roms, (size_t)std::max(s->nroms, 1) * sizeof(RomDev)},
      {A.off_j, sizeof(double)},
      {A.off_rtab, 2 * (size_t)std::max(s->nroms, 1) * sizeof(RomDev)},
      {A.off_dgoff, models ? (size_t)std::max(s->nroms, 1) * sizeof(int64_t) : 0},
      {A.off_dg, A.dg_elems * sizeof(double)}};
  size_t end = 0;
  for (const auto& pt : parts) {
    if (pt[0] < end || pt[0] % 256 != 0) return fail(FDTD_EINVAL, "internal: adjoint workspace parts overlap");
    end = pt[0] + pt[1];
  }
  if (end > A.total) return fail(FDTD_EINVAL, "internal: adjoint workspace parts exceed the total");
  if (A.set_bytes + A.xs_bytes > A.ck_psi || A.ck_psi + (L.pml ? 4 * fb : 0) > A.ck_stride ||
      (L.pml && 5 * fb > A.slot_bytes))
    return fail(FDTD_EINVAL, "internal: checkpoint or slot parts overlap");
  return FDTD_OK;
}

// [p, p + bytes) inside [base, base + total)
bool inside_span(const void* p, size_t bytes, const void* base, size_t total) {
  const uintptr_t a = (uintptr_t)p, b = (uintptr_t)base;
  return a >= b && bytes <= total && a - b <= total - bytes;
}

// Every pointer and extent a recompute launch writes lies in the adjoint
// workspace: the output field set (three field arrays), the private step
// counter, the two images of reduced states it reads and writes (xs +
// x_off + par * xstride with xstride = +img or -img) and its model table;
// its input set lies in the workspace too (a checkpoint or an earlier slot).
template <typename T>
int check_recompute(const StepParams<T>& rp, int par, const char* aw, const AdjLayout& A, size_t fe, int nroms) {
  const size_t fb = fe * sizeof(T);
  for (int f = 0; f < 3; ++f)
    if (!inside_span(rp.f[par][f], fb, aw, A.total) || !inside_span(rp.f[par ^ 1][f], fb, aw, A.total))
      return fail(FDTD_EINVAL, "internal: recompute field %d outside the adjoint workspace", f);
  const char* xlo = (const char*)rp.xs - (par ? A.img * sizeof(T) : 0);
  const char* rec = aw + A.off_xrec;
  bool in_set = false;  // both images inside one buffer set's images
  for (int b = 0; b < A.nbuf; ++b)
    in_set = in_set || inside_span(xlo, 2 * A.img * sizeof(T), rec + b * A.xrec_stride,
                                   (size_t)(A.K + 1) * A.img * sizeof(T));
  if (!inside_span(rp.ctrl, kCtrlInts * sizeof(int), aw, A.total) || !in_set)
    return fail(FDTD_EINVAL, "internal: recompute control or reduced-state images outside the adjoint workspace");
  if (nroms > 0 && !inside_span(rp.roms, (size_t)nroms * sizeof(RomDev), aw + A.off_rtab,
                                2 * (size_t)nroms * sizeof(RomDev)))
    return fail(FDTD_EINVAL, "internal: recompute model table outside the adjoint workspace");
  if (rp.nprobes != 0) return fail(FDTD_EINVAL, "internal: recompute records probes");
  return FDTD_OK;
}

// The reverse sweep.  noalloc: the workspace is the static scratch array
// and nothing is allocated - G^T is transposed on the device from the
// handle's own G (the same FP64-formed, rounded values the host builds),
// the model table is patched on the device, the forward uses plain launches
// (run_direct_any), the objective is summed on the device, scratch is
// cleared by a fill kernel and the gradients are copied straight into the
// caller's arrays.
// Host outputs of the gradients through the models: per region dJ/dR~,
// dJ/dF~ (q x q) and dJ/dL~ (q x np), row-major; null entries are skipped.
struct ModelOut {
  double* const* rt;
  double* const* ft;
  double* const* lt;
};

// Reverse-mode step through the closed form of eq. (23) for one region:
// from dJ/dG (gG, nc x nc row-major, nc = q + np) to dJ/dR~, dJ/dF~,
// dJ/dL~ and to the port half cells C+, C- of eq. (13).  With
// M = R~ + F~ + L~ C+ L~^T, N = R~ - F~ + L~ C- L~^T, A~ = M^{-1} N,
// B~' = M^{-1} L~ Sc, C~ = L~^T and G = [[A~, B~'], [C~A~, C~B~']]:
//   dA~ = gG_xx + C~^T gG_yx,  dB~' = gG_xu + C~^T gG_yu,
//   dC~ = gG_yx A~^T + gG_yu B~'^T,  [W_A | W_B] = M^{-T} [dA~ | dB~'],
//   dN = W_A,  dM = -(W_A A~^T + W_B B~'^T),  dR~ = dM + dN,  dF~ = dM - dN,
//   dL~ = (dM + dM^T) L~ C+ + (dN + dN^T) L~ C- + W_B Sc + dC~^T,
//   dC+_k = l_k^T dM l_k,  dC-_k = l_k^T dN l_k  (l_k column k of L~).
bool model_vjp(const RomHost& h, const std::vector<double>& gG, std::vector<double>& gR, std::vector<double>& gF,
               std::vector<double>& gL, std::vector<double>& gcp, std::vector<double>& gcm) {
  const int q = h.q, np = h.np, nc = q + np;
  auto G = [&](int r, int c) { return gG[(size_t)r * nc + c]; };
  auto Lt = [&](int a, int k) { return h.C[(size_t)k * q + a]; };
  // W = [dA~ | dB~'] (q x nc), then M^{-T} W
  std::vector<double> W((size_t)q * nc), gC((size_t)np * q, 0.0);
  for (int a = 0; a < q; ++a)
    for (int c = 0; c < nc; ++c) {
      double v = G(a, c);
      for (int k = 0; k < np; ++k) v += Lt(a, k) * G(q + k, c);
      W[(size_t)a * nc + c] = v;
    }
  for (int k = 0; k < np; ++k)
    for (int a = 0; a < q; ++a) {
      double v = 0;
      for (int b = 0; b < q; ++b) v += G(q + k, b) * h.A[(size_t)a * q + b];
      for (int c = 0; c < np; ++c) v += G(q + k, q + c) * h.B[(size_t)a * np + c];
      gC[(size_t)k * q + a] = v;
    }
  std::vector<double> MT((size_t)q * q);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      double v = h.R[(size_t)a * q + b] + h.F[(size_t)a * q + b];
      for (int k = 0; k < np; ++k) v += Lt(a, k) * h.cp[k] * Lt(b, k);
      MT[(size_t)b * q + a] = v;
    }
  std::vector<int> piv;
  if (!la::lu_factor(q, MT.data(), piv)) return false;
  la::lu_solve(q, MT.data(), piv, W.data(), nc);
  std::vector<double> gM((size_t)q * q), gN((size_t)q * q);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      double v = 0;
      for (int c = 0; c < q; ++c) v += W[(size_t)a * nc + c] * h.A[(size_t)b * q + c];
      for (int c = 0; c < np; ++c) v += W[(size_t)a * nc + q + c] * h.B[(size_t)b * np + c];
      gM[(size_t)a * q + b] = -v;
      gN[(size_t)a * q + b] = W[(size_t)a * nc + b];
    }
  gR.resize((size_t)q * q);
  gF.resize((size_t)q * q);
  for (size_t e = 0; e < gR.size(); ++e) {
    gR[e] = gM[e] + gN[e];
    gF[e] = gM[e] - gN[e];
  }
  gL.assign((size_t)q * np, 0.0);
  gcp.assign(np, 0.0);
  gcm.assign(np, 0.0);
  for (int k = 0; k < np; ++k) {
    std::vector<double> mp(q, 0.0), mn(q, 0.0);  // (dM + dM^T) l_k, (dN + dN^T) l_k
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < q; ++b) {
        const double l = Lt(b, k);
        if (l == 0.0) continue;
        mp[a] += (gM[(size_t)a * q + b] + gM[(size_t)b * q + a]) * l;
        mn[a] += (gN[(size_t)a * q + b] + gN[(size_t)b * q + a]) * l;
      }
    double sp = 0, sm = 0;
    for (int a = 0; a < q; ++a) {
      gL[(size_t)a * np + k] = mp[a] * h.cp[k] + mn[a] * h.cm[k] + W[(size_t)a * nc + q + k] * h.sc[k] +
                               gC[(size_t)k * q + a];
      sp += Lt(a, k) * mp[a];
      sm += Lt(a, k) * mn[a];
    }
    gcp[k] = 0.5 * sp;  // l^T dM l = l^T (dM + dM^T) l / 2
    gcm[k] = 0.5 * sm;
  }
  return true;
}

template <typename T>
int adjoint_impl(fdtd_rom_sim* s, int N, int probe, char* aw, const AdjLayout& A, double* J,
                 double* grad_eps, double* grad_sig, bool noalloc, const ModelOut* mo = nullptr) {
  const Layout& L = s->L;
  hipStream_t st = s->stream;
  const size_t fe = L.field_elems;
  char* ws = s->ws;
  auto dev_err = [&](const char* what) {
    return fail(FDTD_EDEVICE, "%s failed: %s", what, hipGetErrorString(hipGetLastError()));
  };
  // the slots' padding columns of every buffer set
  auto clear_padding = [&]() {
    for (int b = 0; b < A.nbuf; ++b)
      if (launch_zero_padding<T>((T*)(aw + A.off_slots + b * A.slots_stride),
                                 (size_t)A.K * (A.slot_bytes / (fe * sizeof(T))), s->ny, s->pitch, s->nx,
                                 st) != hipSuccess)
        return false;
    return true;
  };
  if (noalloc) {
    // clear the control block, everything from the recompute's psi at Hz to
    // G^T and the slots' padding columns, as the host path below does
    if (launch_zero_fill(aw + A.off_ctrl, align_up(kCtrlInts * sizeof(int), 16), st) != hipSuccess ||
        launch_zero_fill(aw + A.off_psih, A.off_gt - A.off_psih, st) != hipSuccess || !clear_padding())
      return dev_err("scratch clear");
    const T* mats = (const T*)(ws + L.off_mats);
    T* gt = (T*)(aw + A.off_gt);
    for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
      const RomHost& h = s->roms[L.slot_rep[sl]];
      const int nc = h.q + h.np;
      if (launch_transpose_block<T>(mats + L.slot_off[sl], gt + slot_gt(s, sl), (int)align_up((size_t)nc, kWave), nc,
                                    st) != hipSuccess)
        return dev_err("G^T transpose");
    }
    const RomDev* rin = (const RomDev*)(ws + L.off_roms);
    RomDev* rout = (RomDev*)(aw + A.off_roms);
    for (int k = 0; k < s->nroms; ++k)
      if (launch_rom_entry(rout + k, rin + k, (int64_t)slot_gt(s, L.slot_of_rom[k]), st) != hipSuccess)
        return dev_err("model table");
  } else {
    // G^T of every matrix slot (row k = column k of eq. (23)'s G) and the
    // model table pointing at it
    std::vector<T> gt(std::max<size_t>(A.gt_elems, 1), T(0));
    for (size_t sl = 0; sl < L.slot_rep.size(); ++sl) {
      const RomHost& h = s->roms[L.slot_rep[sl]];
      const int q = h.q, np = h.np;
      const size_t ldg = align_up((size_t)q + np, kWave);
      std::vector<double> CA((size_t)np * q), CB((size_t)np * np);
      la::gemm(np, q, q, h.C.data(), h.A.data(), CA.data());
      la::gemm(np, np, q, h.C.data(), h.B.data(), CB.data());
      T* g = gt.data() + slot_gt(s, sl);
      auto put = [&](int row, int col, double v) { g[(size_t)col * ldg + row] = (T)v; };
      for (int a = 0; a < q; ++a) {
        for (int c = 0; c < q; ++c) put(a, c, h.A[(size_t)a * q + c]);
        for (int c = 0; c < np; ++c) put(a, q + c, h.B[(size_t)a * np + c]);
      }
      for (int k = 0; k < np; ++k) {
        for (int c = 0; c < q; ++c) put(q + k, c, CA[(size_t)k * q + c]);
        for (int c = 0; c < np; ++c) put(q + k, q + c, CB[(size_t)k * np + c]);
      }
    }
    std::vector<RomDev> rd(s->nroms);
    for (int k = 0; k < s->nroms; ++k) {
      const RomHost& h = s->roms[k];
      rd[k].q = h.q;
      rd[k].np = h.np;
      rd[k].n_ex = 2 * h.ni;
      rd[k].ldg = (int)align_up((size_t)h.q + h.np, kWave);
      rd[k].g_off = -1;
      rd[k].x_off = (int64_t)L.x_off[k];
      rd[k].xstride = (int64_t)align_up((size_t)h.q, 64);
      rd[k].i_off = (int64_t)L.i_off[k];
      rd[k].gt_off = (int64_t)slot_gt(s, L.slot_of_rom[k]);
    }
    if (hipMemcpyAsync(aw + A.off_gt, gt.data(), A.gt_elems * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess ||
        (s->nroms > 0 && hipMemcpyAsync(aw + A.off_roms, rd.data(), rd.size() * sizeof(RomDev),
                                        hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
      return dev_err("model upload");
    // zero the private step counter; the recompute's psi at Hz (only waves
    // that reach a layer write it, the rest of it must read zero), the
    // adjoint fields, states and gradients; and the slots' padding columns
    // (the stencil reads them unguarded and never writes them - every other
    // sample of a slot is written by its recompute step before it is read)
    if (hipMemsetAsync(aw + A.off_ctrl, 0, kCtrlInts * sizeof(int), st) != hipSuccess ||
        hipMemsetAsync(aw + A.off_psih, 0, A.off_gt - A.off_psih, st) != hipSuccess || !clear_padding())
      return dev_err("workspace clear");
    if (A.models && s->nroms > 0) {
      std::vector<int64_t> dgo(s->nroms);
      for (int k = 0; k < s->nroms; ++k) dgo[k] = (int64_t)region_dg(s, k);
      if (hipMemsetAsync(aw + A.off_dg, 0, A.dg_elems * sizeof(double), st) != hipSuccess ||
          hipMemcpyAsync(aw + A.off_dgoff, dgo.data(), dgo.size() * sizeof(int64_t), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return dev_err("model gradient set-up");
    }
  }
  // the recompute's model tables: the handle's, with xstride = +img, -img
  const RomDev* hroms = (const RomDev*)(ws + L.off_roms);
  RomDev* rtab = (RomDev*)(aw + A.off_rtab);
  if (launch_rom_xstride(rtab, hroms, s->nroms, (int64_t)A.img, st) != hipSuccess ||
      launch_rom_xstride(rtab + s->nroms, hroms, s->nroms, -(int64_t)A.img, st) != hipSuccess)
    return dev_err("recompute model tables");

  auto ckpt = [&](int c) { return aw + A.off_ckpt + (size_t)c * A.ck_stride; };
  auto ckpt_xs = [&](int c) { return ckpt(c) + align_up(A.set_bytes, 256); };
  // checkpoint's auxiliary fields: [psi at Hz (2), psi at Ex, psi at Ey]
  auto ckpt_psi = [&](int c) { return (T*)(ckpt(c) + A.ck_psi); };
  // segment c's buffer set of slots and images (segments alternate when the
  // recompute of the segment below runs beside the reverse steps)
  auto bset = [&](int c) -> size_t { return A.nbuf == 2 ? (size_t)(c & 1) : 0; };
  auto slot = [&](int c, int k) { return aw + A.off_slots + bset(c) * A.slots_stride + (size_t)k * A.slot_bytes; };
  // reduced states x~^{m0+k} of segment c, k = 0..K
  auto image = [&](int c, int k) { return (T*)(aw + A.off_xrec + bset(c) * A.xrec_stride) + (size_t)k * A.img; };
  // state m0 + k of segment c: k = 0 is the checkpoint, k >= 1 is slot k - 1
  auto state = [&](int c, int k) -> T* { return (T*)(k == 0 ? ckpt(c) : slot(c, k - 1)); };
  // psi at Ex then at Ey of state m0 + k (contiguous)
  auto psi_e = [&](int c, int k) -> T* { return k == 0 ? ckpt_psi(c) + 2 * fe : state(c, k) + 3 * fe; };
  T* psih = (T*)(aw + A.off_psih);  // recompute's psi at Hz, [parity][2]
  const size_t xs_copy = L.xs_elems * sizeof(T);
  const size_t fb = fe * sizeof(T);
  const StepParams<T>& sp = step_params<T>(s);

  // forward with checkpoints; the last segment's steps are not taken here:
  // its recompute takes them and hands the handle the result
  for (int c = 0; c < A.nck; ++c) {
    const int m0 = c * A.K;
    const int len = std::min(A.K, N - m0);
    const char* cur = ws + L.off_fields + (size_t)cur_set(s) * A.set_bytes;
    if (hipMemcpyAsync(ckpt(c), cur, A.set_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        (xs_copy > 0 && hipMemcpyAsync(ckpt_xs(c), ws + L.off_xs, xs_copy, hipMemcpyDeviceToDevice, st) != hipSuccess))
      return dev_err("checkpoint copy");
    if (L.pml) {
      const T* src[4] = {sp.psi_h[m0 & 1][0], sp.psi_h[m0 & 1][1], sp.psi_ex, sp.psi_ey};
      for (int k = 0; k < 4; ++k)
        if (hipMemcpyAsync(ckpt_psi(c) + k * fe, src[k], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
          return dev_err("checkpoint copy");
    }
    if (c == A.nck - 1) break;
    const int rc = noalloc ? run_direct_any(s, len) : run_steps_any(s, len);
    if (rc != FDTD_OK) return rc;
  }

  // objective from the probe record (once the last segment has filled it)
  auto objective = [&]() -> int {
    if (noalloc) {
      double* jd = (double*)(aw + A.off_j);
      if (launch_probe_energy<T>((const T*)(ws + L.off_pbuf), s->nprobes, probe, N, s->dt, jd, st) != hipSuccess ||
          hipMemcpyAsync(J, jd, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return dev_err("objective");
      if (!std::isfinite(*J)) return fail(FDTD_EUNSTABLE, "non-finite objective");
      return FDTD_OK;
    }
    return fdtd_rom_probe_objective(s, probe, 0, N, J);
  };

  // reverse sweep
  StepParams<T> rp = step_params<T>(s);
  rp.ctrl = (int*)(aw + A.off_ctrl);
  rp.nprobes = 0;
  AdjParams<T> ap{};
  ap.al = sp.al;
  ap.be = sp.be;
  ap.mi = sp.mi;
  ap.mt = sp.mt;
  ap.midx = sp.midx;
  double* g64 = (double*)(aw + A.off_g);
  // FP32: the gradients are summed in FP32 over at most kFoldSteps steps
  // (folded into g64 at every multiple of kFoldSteps and at every
  // checkpoint), so their rounding does not grow with the checkpoint interval
  constexpr bool kSeg = sizeof(T) == 4;
  constexpr int kFoldSteps = 128;
  if constexpr (kSeg) {
    ap.ga_e = (T*)(aw + A.off_gseg);
  } else {
    ap.ga_e = (T*)g64;
  }
  ap.ga_s = ap.ga_e + fe;
  ap.nx = s->nx;
  ap.ny = s->ny;
  ap.pitch = s->pitch;
  // rows per reverse wave: the forward's default, at most 16 (the C5 1024^2
  // sweep with the stream tiles in XCD runs: 117.5 ms at 4 rows, 131.0 at
  // 2, 137.0 at 8 with the recompute beside the reverse steps; 111.0, 117.3
  // and 126.4 ms with every state resident)
  ap.seg = std::min(default_tiling(s->nx, s->ny, (int)L.tsize), 16);
  ap.chdy = sp.chdy;
  ap.chdx = sp.chdx;
  ap.k2dy = sp.k2dy;
  ap.k2dx = sp.k2dx;
  ap.dx = s->dx;
  ap.dy = s->dy;
  ap.fa = kEps0 / (2.0 * s->dt);
  ap.obj_off = (int64_t)s->probes[probe].j * s->pitch + s->probes[probe].i;
  ap.obj_coef = (T)(2.0 * s->dt);
  ap.roms = (const RomDev*)(aw + A.off_roms);
  ap.blocks = (const RowBlock*)(ws + L.off_blocks);
  ap.nblocks = s->nroms > 0 ? L.nrowblocks : 0;
  ap.mats = (const T*)(aw + A.off_gt);
  ap.idx = (const int*)(ws + L.off_idx);
  ap.pml = L.pml ? 1 : 0;
  ap.dgt = A.models && s->nroms > 0 ? (double*)(aw + A.off_dg) : nullptr;
  ap.dg_off = (const int64_t*)(aw + A.off_dgoff);
  ap.pml_xlo = sp.pml_xlo;
  ap.pml_xhi = sp.pml_xhi;
  ap.pml_ylo = sp.pml_ylo;
  ap.pml_yhi = sp.pml_yhi;
  ap.px_stride = sp.px_stride;
  ap.py_stride = sp.py_stride;
  ap.px = sp.px;
  ap.py = sp.py;
  T* lam[2] = {(T*)(aw + A.off_lam), (T*)(aw + A.off_lam + A.lam_bytes)};
  T* lx[2] = {(T*)(aw + A.off_lx), (T*)(aw + A.off_lx + A.xs_bytes)};
  T* pend[2] = {(T*)(aw + A.off_pend), (T*)(aw + A.off_pend + fb)};
  // recompute of segment c on stream qs: states m0+1 .. m0+len into its
  // slots 0 .. len-1, reduced states into its images
  auto recompute = [&](int c, hipStream_t qs) -> int {
    const int m0 = c * A.K;
    const int len = std::min(A.K, N - m0);
    if (launch_states_to_image<T>((const T*)ckpt_xs(c), image(c, 0), hroms, s->nroms, m0 & 1, qs) != hipSuccess)
      return dev_err("state restore");
    if (L.pml && hipMemcpyAsync(psih + (size_t)(m0 & 1) * 2 * fe, ckpt_psi(c), 2 * fb, hipMemcpyDeviceToDevice,
                                qs) != hipSuccess)
      return dev_err("state restore");
    for (int k = 0; k < len; ++k) {  // states m0+1 .. m0+len into slots 0 .. len-1
      const int m = m0 + k;
      const int par = m & 1;
      T* in = state(c, k);
      T* out = state(c, k + 1);
      for (int f = 0; f < 3; ++f) {
        rp.f[par][f] = in + (size_t)f * fe;
        rp.f[par ^ 1][f] = out + (size_t)f * fe;
      }
      if (L.pml) {
        // the step updates psi at Ex and Ey in place: start the new slot's
        // pair from this state's
        if (hipMemcpyAsync(psi_e(c, k + 1), psi_e(c, k), 2 * fb, hipMemcpyDeviceToDevice, qs) != hipSuccess)
          return dev_err("recompute copy");
        for (int q = 0; q < 2; ++q) {
          rp.psi_h[q][0] = psih + (size_t)q * 2 * fe;
          rp.psi_h[q][1] = psih + (size_t)q * 2 * fe + fe;
        }
        rp.psi_ex = psi_e(c, k + 1);
        rp.psi_ey = psi_e(c, k + 1) + fe;
      }
      rp.step_off = m;
      rp.roms = par ? rtab + s->nroms : rtab;
      rp.xs = par ? image(c, k + 1) : image(c, k);
      if (const int rc = check_recompute<T>(rp, par, aw, A, fe, s->nroms); rc != FDTD_OK) return rc;
      if (launch_step<T>(rp, s->seg, s->smem, qs) != hipSuccess) return dev_err("recompute launch");
    }
    return FDTD_OK;
  };
  // the recompute of segment c-1 runs on a second stream (default priority)
  // beside the reverse steps of segment c; events order it after the
  // reverse steps of segment c+1, whose buffer set it takes over
  struct Pipe {
    hipStream_t sb = nullptr;
    hipEvent_t ev[5] = {};  // start, recomputed[2], reversed[2]
    ~Pipe() {
      if (sb) (void)hipStreamSynchronize(sb);
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      if (sb) (void)hipStreamDestroy(sb);
    }
  } pipe;
  const bool piped = A.nbuf == 2 && !noalloc;
  if (piped) {
    if (hipStreamCreateWithFlags(&pipe.sb, hipStreamNonBlocking) != hipSuccess) return dev_err("recompute stream");
    for (hipEvent_t& e : pipe.ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return dev_err("recompute events");
  }
  hipEvent_t& ev_start = pipe.ev[0];
  hipEvent_t* ev_rec = pipe.ev + 1;
  hipEvent_t* ev_rev = pipe.ev + 3;
  int cur = 0;
  for (int c = A.nck - 1; c >= 0; --c) {
    const int m0 = c * A.K;
    const int len = std::min(A.K, N - m0);
    if (!piped || c == A.nck - 1) {
      if (const int rc = recompute(c, st); rc != FDTD_OK) return rc;
    } else if (hipStreamWaitEvent(st, ev_rec[c & 1], 0) != hipSuccess) {
      return dev_err("recompute wait");
    }
    if (c == A.nck - 1) {
      // the forward stopped at m0: the handle takes the recomputed state
      // after step N (fields into its set for N, reduced states into their
      // parity-N places, with layers the auxiliary fields), the segment's
      // probe rows and the step count, as if it had run the steps
      const int dst = (N & 1) ^ s->flip;
      if (hipMemcpyAsync(ws + L.off_fields + (size_t)dst * A.set_bytes, state(c, len), A.set_bytes,
                         hipMemcpyDeviceToDevice, st) != hipSuccess ||
          launch_image_to_states<T>(image(c, len), (T*)(ws + L.off_xs), hroms, s->nroms, N & 1, st) != hipSuccess)
        return dev_err("handing over the last segment");
      if (L.pml) {
        const T* ph = psih + (size_t)(N & 1) * 2 * fe;
        if (hipMemcpyAsync(sp.psi_h[N & 1][0], ph, fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(sp.psi_h[N & 1][1], ph + fe, fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(sp.psi_ex, psi_e(c, len), fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(sp.psi_ey, psi_e(c, len) + fe, fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
          return dev_err("handing over the last segment");
      }
      if (launch_slots_to_probes<T>(state(c, 1), A.slot_bytes / sizeof(T), fe, len, s->nprobes, sp.probe_off,
                                    sp.probe_comp, sp.probe_buf, m0, st) != hipSuccess ||
          launch_tick(sp.ctrl, len, st) != hipSuccess)
        return dev_err("handing over the last segment");
      s->steps = N;
      if (const int rc = objective(); rc != FDTD_OK) return rc;
    }
    if (piped && c >= 1) {
      // after the hand-over (the recompute's private psi at Hz is free), or
      // once segment c+1's reverse steps have left its buffer set
      if (c == A.nck - 1 && hipEventRecord(ev_start, st) != hipSuccess) return dev_err("recompute event");
      if (hipStreamWaitEvent(pipe.sb, c == A.nck - 1 ? ev_start : ev_rev[(c + 1) & 1], 0) != hipSuccess)
        return dev_err("recompute wait");
      if (const int rc = recompute(c - 1, pipe.sb); rc != FDTD_OK) return rc;
      if (hipEventRecord(ev_rec[(c - 1) & 1], pipe.sb) != hipSuccess) return dev_err("recompute event");
    }
    for (int k = len - 1; k >= 0; --k) {
      T* li = lam[cur];
      T* lo = lam[cur ^ 1];
      ap.lhz_in = li;
      ap.lex_in = li + fe;
      ap.ley_in = li + 2 * fe;
      ap.lhz_out = lo;
      ap.lex_out = lo + fe;
      ap.ley_out = lo + 2 * fe;
      ap.lx_in = lx[cur];
      ap.lx_out = lx[cur ^ 1];
      ap.hz1 = state(c, k + 1);
      ap.xn = image(c, k);
      ap.ex0 = state(c, k) + fe;
      ap.ey0 = state(c, k) + 2 * fe;
      if (L.pml) {
        for (int q = 0; q < 4; ++q) {
          ap.lps_in[q] = li + (size_t)(3 + q) * fe;
          ap.lps_out[q] = lo + (size_t)(3 + q) * fe;
        }
        ap.pex1 = psi_e(c, k + 1);
        ap.pey1 = psi_e(c, k + 1) + fe;
      }
      if (A.models) {
        // two launches: eq. (23)'s transpose of step m (accumulating dJ/dG
        // with this segment's x~^m), then the stream
        if (launch_adjoint_step<T>(ap, L.smem_gemv, st) != hipSuccess) return dev_err("adjoint launch");
      } else {
        // one launch: the stream of step m with lambda_h^m from the launch
        // before, and eq. (23)'s transpose of step m-1 (none for m = 0)
        ap.pend_in = pend[cur];
        ap.pend_out = pend[cur ^ 1];
        if (launch_adjoint_fused<T>(ap, m0 + k >= 1, L.smem_gemv, st) != hipSuccess)
          return dev_err("adjoint launch");
      }
      cur ^= 1;
      if constexpr (kSeg) {
        if ((k == 0 || (m0 + k) % kFoldSteps == 0) &&
            launch_adjoint_flush((float*)ap.ga_e, g64, 2 * fe, st) != hipSuccess)
          return dev_err("gradient flush");
      }
    }
    if (piped && hipEventRecord(ev_rev[c & 1], st) != hipSuccess) return dev_err("reverse event");
  }
  // gradients: pitch layout -> natural, zero on regions and their rings and
  // on PEC cells
  const int nx = s->nx, ny = s->ny, P = s->pitch;
  const double* gd = (const double*)(aw + A.off_g);
  if (noalloc) {
    // straight into the caller's arrays, row by row
    if (hipMemcpy2DAsync(grad_eps, (size_t)nx * sizeof(double), gd, (size_t)P * sizeof(double),
                         (size_t)nx * sizeof(double), ny, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpy2DAsync(grad_sig, (size_t)nx * sizeof(double), gd + fe, (size_t)P * sizeof(double),
                         (size_t)nx * sizeof(double), ny, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return dev_err("gradient read");
  } else {
    // one contiguous copy (much faster than rows into pageable memory)
    std::vector<double> g(2 * fe);
    if (hipMemcpyAsync(g.data(), gd, 2 * fe * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return dev_err("gradient read");
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        grad_eps[(size_t)j * nx + i] = g[(size_t)j * P + i];
        grad_sig[(size_t)j * nx + i] = g[fe + (size_t)j * P + i];
      }
  }
  for (size_t c = 0; c < s->pec.size(); ++c)
    if (s->pec[c]) grad_eps[c] = grad_sig[c] = 0.0;  // metal: no material gradient
  // regions (and, with the models held, their rings) report zero
  const int ring = A.models ? 0 : 1;
  for (const RomHost& h : s->roms)
    for (int j = std::max(h.j0 - ring, 0); j < std::min(h.j0 + h.nj + ring, ny); ++j)
      for (int i = std::max(h.i0 - ring, 0); i < std::min(h.i0 + h.ni + ring, nx); ++i)
        grad_eps[(size_t)j * nx + i] = grad_sig[(size_t)j * nx + i] = 0.0;
  if (A.models && s->nroms > 0) {
    // dJ/dG^T per region -> dJ/dG -> the closed form's inputs; the port half
    // cells' share goes to the ring cells: C+- = Dl Dl' (eps0 eps_r/dt +- sigma/2)
    std::vector<double> dgt(A.dg_elems);
    if (hipMemcpyAsync(dgt.data(), aw + A.off_dg, A.dg_elems * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return dev_err("model gradient read");
    for (int k = 0; k < s->nroms; ++k) {
      const RomHost& h = s->roms[k];
      const int q = h.q, np = h.np, nc = q + np;
      const size_t ldg = align_up((size_t)nc, kWave);
      const double* d = dgt.data() + region_dg(s, k);
      std::vector<double> gG((size_t)nc * nc), gR, gF, gL, gcp, gcm;
      for (int r = 0; r < nc; ++r)
        for (int c = 0; c < nc; ++c) gG[(size_t)r * nc + c] = d[(size_t)c * ldg + r];
      if (!model_vjp(h, gG, gR, gF, gL, gcp, gcm))
        return fail(FDTD_ENOTPASSIVE, "region %d: eq. (23) matrix M is singular", k);
      for (int c = 0; c < np; ++c) {
        int oi, oj;
        double dl, dlh;
        if (c < h.ni) { oi = h.i0 + c; oj = h.j0 - 1; dl = s->dx; dlh = s->dy / 2; }
        else if (c < 2 * h.ni) { oi = h.i0 + c - h.ni; oj = h.j0 + h.nj; dl = s->dx; dlh = s->dy / 2; }
        else if (c < 2 * h.ni + h.nj) { oi = h.i0 - 1; oj = h.j0 + c - 2 * h.ni; dl = s->dy; dlh = s->dx / 2; }
        else { oi = h.i0 + h.ni; oj = h.j0 + c - 2 * h.ni - h.nj; dl = s->dy; dlh = s->dx / 2; }
        const size_t ci = (size_t)oj * nx + oi;
        if (!s->pec.empty() && s->pec[ci]) continue;
        grad_eps[ci] += dl * dlh * kEps0 / s->dt * (gcp[c] + gcm[c]);
        grad_sig[ci] += dl * dlh * 0.5 * (gcp[c] - gcm[c]);
      }
      if (mo->rt && mo->rt[k]) std::copy(gR.begin(), gR.end(), mo->rt[k]);
      if (mo->ft && mo->ft[k]) std::copy(gF.begin(), gF.end(), mo->ft[k]);
      if (mo->lt && mo->lt[k]) std::copy(gL.begin(), gL.end(), mo->lt[k]);
    }
  }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t c = (size_t)j * nx + i;
      if (!std::isfinite(grad_eps[c]) || !std::isfinite(grad_sig[c]))
        return fail(FDTD_EUNSTABLE, "non-finite gradient at cell (%d,%d)", i, j);
    }
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_rom_adjoint_workspace_size(const fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every,
                                    size_t* bytes) {
  if (!sim || !bytes) return fail(FDTD_EINVAL, "null argument");
  try {
    AdjLayout A;
    const int rc = plan_adjoint(sim, nsteps, ckpt_every, A);
    if (rc != FDTD_OK) return rc;
    *bytes = A.total;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_adjoint(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe,
                     void* dev_adj_ws, size_t ws_bytes, double* J, double* grad_eps_r,
                     double* grad_sigma) {
  if (!sim || !J || !grad_eps_r || !grad_sigma) return fail(FDTD_EINVAL, "null argument");
  if (sim->steps != 0) return fail(FDTD_ESTATE, "the adjoint starts from the initial state (%d steps taken)", sim->steps);
  if (probe < 0 || probe >= sim->nprobes) return fail(FDTD_EINVAL, "probe %d out of range", probe);
  if (sim->probes[probe].comp != FDTD_HZ) return fail(FDTD_EINVAL, "probe %d is not an Hz probe", probe);
  try {
    AdjLayout A;
    int rc = plan_adjoint(sim, nsteps, ckpt_every, A);
    if (rc != FDTD_OK) return rc;
    if (!dev_adj_ws) return fail(FDTD_EINVAL, "null adjoint workspace");
    if (((uintptr_t)dev_adj_ws) % 256) return fail(FDTD_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (ws_bytes < A.total) return fail(FDTD_ENOMEM, "adjoint workspace has %zu bytes, %zu needed", ws_bytes, A.total);
    char* aw = (char*)dev_adj_ws;
    return sim->dtype == FDTD_F32 ? adjoint_impl<float>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, false)
                                  : adjoint_impl<double>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, false);
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_adjoint_models_workspace_size(const fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every,
                                           size_t* bytes) {
  if (!sim || !bytes) return fail(FDTD_EINVAL, "null argument");
  try {
    AdjLayout A;
    const int rc = plan_adjoint(sim, nsteps, ckpt_every, A, true);
    if (rc != FDTD_OK) return rc;
    *bytes = A.total;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_adjoint_models(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe,
                            void* dev_adj_ws, size_t ws_bytes, double* J, double* grad_eps_r,
                            double* grad_sigma, double* const* grad_Rt, double* const* grad_Ft,
                            double* const* grad_Lt) {
  if (!sim || !J || !grad_eps_r || !grad_sigma) return fail(FDTD_EINVAL, "null argument");
  if (sim->steps != 0) return fail(FDTD_ESTATE, "the adjoint starts from the initial state (%d steps taken)", sim->steps);
  if (probe < 0 || probe >= sim->nprobes) return fail(FDTD_EINVAL, "probe %d out of range", probe);
  if (sim->probes[probe].comp != FDTD_HZ) return fail(FDTD_EINVAL, "probe %d is not an Hz probe", probe);
  try {
    AdjLayout A;
    int rc = plan_adjoint(sim, nsteps, ckpt_every, A, true);
    if (rc != FDTD_OK) return rc;
    if (!dev_adj_ws) return fail(FDTD_EINVAL, "null adjoint workspace");
    if (((uintptr_t)dev_adj_ws) % 256) return fail(FDTD_EINVAL, "adjoint workspace must be 256-byte aligned");
    if (ws_bytes < A.total) return fail(FDTD_ENOMEM, "adjoint workspace has %zu bytes, %zu needed", ws_bytes, A.total);
    char* aw = (char*)dev_adj_ws;
    const ModelOut mo{grad_Rt, grad_Ft, grad_Lt};
    return sim->dtype == FDTD_F32
               ? adjoint_impl<float>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, false, &mo)
               : adjoint_impl<double>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, false, &mo);
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_adjoint_plan(const fdtd_problem* prob, int32_t nsteps, int32_t ckpt_every, size_t* bytes) {
  if (!prob || !bytes) return fail(FDTD_EINVAL, "null argument");
  try {
    // a host-only stand-in for the handle: the layout and the model shapes
    fdtd_rom_sim s;
    int rc = plan_problem(prob, s.L);
    if (rc != FDTD_OK) return rc;
    s.dtype = prob->grid.dtype;
    s.nx = prob->grid.nx;
    s.ny = prob->grid.ny;
    s.max_steps = prob->max_steps;
    s.nroms = prob->nroms;
    s.roms.resize(prob->nroms);
    for (int k = 0; k < prob->nroms; ++k) {
      s.roms[k].q = prob->roms[k].q;
      s.roms[k].np = ports_of(prob->roms[k]);
    }
    AdjLayout A;
    rc = plan_adjoint(&s, nsteps, ckpt_every, A);
    if (rc != FDTD_OK) return rc;
    *bytes = A.total;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_adjoint_noalloc(fdtd_rom_sim* sim, int32_t nsteps, int32_t ckpt_every, int32_t probe, double* J,
                             double* grad_eps_r, double* grad_sigma) {
  if (!sim || !J || !grad_eps_r || !grad_sigma) return fail(FDTD_EINVAL, "null argument");
  if (sim->steps != 0) return fail(FDTD_ESTATE, "the adjoint starts from the initial state (%d steps taken)", sim->steps);
  if (probe < 0 || probe >= sim->nprobes) return fail(FDTD_EINVAL, "probe %d out of range", probe);
  if (sim->probes[probe].comp != FDTD_HZ) return fail(FDTD_EINVAL, "probe %d is not an Hz probe", probe);
  AdjLayout A;
  int rc = plan_adjoint(sim, nsteps, ckpt_every, A, false, false);  // one stream, one buffer set
  if (rc != FDTD_OK) return rc;
  if (A.total > kNoAllocScratchBytes)
    return fail(FDTD_ENOMEM, "the sweep needs %zu bytes of scratch, the static scratch array holds %zu "
                "(use fdtd_rom_adjoint with a workspace)", A.total, kNoAllocScratchBytes);
  void* scr = nullptr;
  if ((rc = noalloc_scratch(&scr)) != FDTD_OK) return rc;
  char* aw = (char*)scr;
  return sim->dtype == FDTD_F32 ? adjoint_impl<float>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, true)
                                : adjoint_impl<double>(sim, nsteps, probe, aw, A, J, grad_eps_r, grad_sigma, true);
}

}  // extern "C"
