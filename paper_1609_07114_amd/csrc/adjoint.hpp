// Parameters of one reverse (adjoint) step; shared by adjoint.hip and the
// host orchestration in adjoint_rt.cpp.
#pragma once

#include "common.hpp"

namespace fdtd {

// Adjoint variables share the forward field layout (pitch, ownership: a
// cell holds the adjoint of its Hz, south Ex and west Ey).  "in" holds the
// adjoint of the state after step n+1, "out" receives that of the state
// after step n.  lhz_in is updated in place by the coupling transpose.
template <typename T>
struct AdjParams {
  T* lhz_in;
  const T* lex_in;
  const T* ley_in;
  T* lhz_out;
  T* lex_out;
  T* ley_out;
  const T* lx_in;    // adjoint reduced states, indexed by RomDev::x_off
  T* lx_out;
  const T* hz1;      // forward Hz^{n+1/2}
  const T* ex0;      // forward E^n
  const T* ey0;
  const T* al;       // per-cell eps0*eps_r/dt (negative inside regions)
  const T* be;       // per-cell sigma/2
  // the same pairs as a 16-bit index per cell into a table of (a, b), when
  // the handle has one (midx = 1): the streamed reverse step then reads 2 B
  // of material per cell instead of 2 x sizeof(T)
  const uint16_t* mi;
  const MatPair<T>* mt;
  int midx;
  // dJ/deps_r and dJ/dsigma accumulators per cell (pitch layout) in the
  // run's precision: the FP64 totals themselves in FP64 runs; in FP32 runs
  // sums over at most 128 steps, folded into the FP64 totals at every
  // multiple of 128 steps and at every checkpoint (adj_flush)
  T* ga_e;
  T* ga_s;
  int nx, ny, pitch;
  int seg;           // rows per wave of the streamed reverse step (2, 4, 8, 16)
  T chdy, chdx, k2dy, k2dx;
  double dx, dy;
  double fa;         // d(eps0*eps_r/dt averaged on an edge)/d eps_r(cell) = eps0/(2 dt)
  int64_t obj_off;   // Hz sample of the objective
  T obj_coef;        // 2 dt
  // coupling transpose: G^T row-major (RomDev::gt_off), row blocks of kind 0
  const RomDev* roms;
  const RowBlock* blocks;
  int nblocks;
  const T* mats;
  const int* idx;
  // absorbing layers (pml == 0: none): profiles and extents as in
  // StepParams; adjoints of the four auxiliary fields [psi at Hz (d/dx of
  // Ey, d/dy of Ex), psi at Ex, psi at Ey], in/out like the fields; the
  // forward auxiliary fields at Ex and Ey after step n+1
  int pml;
  int pml_xlo, pml_xhi, pml_ylo, pml_yhi;
  int px_stride, py_stride;
  const T* px;
  const T* py;
  const T* lps_in[4];
  T* lps_out[4];
  const T* pex1;
  const T* pey1;
  // gradients through the models (dgt != nullptr): per region k an FP64
  // accumulator of dJ/dG^T at dgt + dg_off[k] (row c = column c of eq.
  // (23)'s G, ldg entries), summed over the steps as
  // [x~^n; h^{n+1/2}]_c [x~^{n+1}; y^{n+1}]-adjoint; xn holds the forward
  // reduced states x~^n at each region's x_off
  double* dgt;
  const int64_t* dg_off;
  const T* xn;
  // fused reverse step (launch_adjoint_fused): lambda_h of eq. (23)'s
  // transpose kept per ring cell in a field-shaped array instead of being
  // added into lhz_in - pend_in holds this step's (added at ring cells by
  // the stream), pend_out receives the step before's (written by the
  // coupling blocks of the same launch); null in the two-launch form
  const T* pend_in;
  T* pend_out;
};

template <typename T>
hipError_t launch_adjoint_step(const AdjParams<T>& p, size_t smem, hipStream_t s);
// One launch per reverse step: the stream of step n (lambda_h of step n in
// pend_in) and, when `coupling`, eq. (23)'s transpose of step n-1, whose
// input adjoint y^n on the interface edges it forms from step n's inputs
// exactly as the stream forms it (lx_in: lambda_x^n, lx_out: lambda_x^{n-1},
// pend_out: lambda_h^{n-1}).  No model-gradient accumulation (dgt null).
template <typename T>
hipError_t launch_adjoint_fused(const AdjParams<T>& p, bool coupling, size_t smem, hipStream_t s);
// g[k] += a[k], a[k] = 0 for k < n (both accumulator pairs: a, g hold 2n)
hipError_t launch_adjoint_flush(float* a, double* g, size_t n, hipStream_t s);

// Pieces of the reverse sweep that runs without allocating
// (fdtd_rom_adjoint_noalloc): its workspace is a file-scope device array of
// kNoAllocScratchBytes per GPU.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
// Device address of the scratch array on the current device (resolved once
// per device with hipGetSymbolAddress and kept).
int noalloc_scratch(void** ptr);
// One ldg x ldg block of G^T (row c = column c of G, zero beyond nc) from
// G (row-major, row length ldg, nc rows).
template <typename T>
hipError_t launch_transpose_block(const T* g, T* gt, int ldg, int nc, hipStream_t s);
// out = in with g_off = -1 and gt_off replaced (one model's table entry).
hipError_t launch_rom_entry(RomDev* out, const RomDev* in, int64_t gt_off, hipStream_t s);
// *out = dt * sum_{k < n} buf[k * nprobes + probe]^2 (FP64, fixed order).
template <typename T>
hipError_t launch_probe_energy(const T* buf, int nprobes, int probe, int n, double dt, double* out,
                               hipStream_t s);
// Zero `bytes` bytes at p (both multiples of 16).
hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s);
// Zero the padding columns [nx, pitch) of `count` consecutive field-shaped
// arrays (ny rows of pitch elements each) starting at base.
template <typename T>
hipError_t launch_zero_padding(T* base, size_t count, int ny, int pitch, int nx, hipStream_t s);

// Forward reduced states kept per step while a segment is recomputed: the
// image of step k holds every region's x~ at its x_off (the parity-0 place
// of the handle's layout).  The recompute's model tables are the handle's
// with xstride = +img (even steps: read image k at rp.xs = image k, write
// image k+1) or -img (odd steps: rp.xs = image k+1), so the step kernel's
// parity addressing lands on consecutive images.
// out[k] = in[k] with xstride replaced, k < nroms.
hipError_t launch_rom_xstride(RomDev* out, const RomDev* in, int nroms, int64_t xstride, hipStream_t s);
// dst[x_off + a] = src[x_off + par * xstride + a] for every region (a < q):
// a checkpoint's states into the parity-0 places of an image.
template <typename T>
hipError_t launch_states_to_image(const T* src, T* dst, const RomDev* roms, int nroms, int par, hipStream_t s);
// The reverse: dst[x_off + par * xstride + a] = src[x_off + a].
template <typename T>
hipError_t launch_image_to_states(const T* src, T* dst, const RomDev* roms, int nroms, int par, hipStream_t s);
// Probe record rows [m0, m0 + len) from recomputed slots (slot k holds the
// state after step m0 + k, fields Hz, Ex, Ey of fe elements each, slots
// `stride` elements apart): buf[(m0 + k) * nprobes + t] = field
// comp[t] of slot k at off[t].
template <typename T>
hipError_t launch_slots_to_probes(const T* slot0, size_t stride, size_t fe, int len, int nprobes, const int* off,
                                  const int* comp, T* buf, int m0, hipStream_t s);

}  // namespace fdtd
