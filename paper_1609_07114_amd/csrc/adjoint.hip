// gfx950 kernels of the reverse (adjoint) sweep for the objective
//   J = dt * sum_n (Hz_p^{n+1/2})^2,
// the transpose of one forward step (eq. (23) coupling, eq. (3) E update,
// eq. (5) H update) applied in reverse order:
//   adj_coupling : [lambda_x~^n; lambda_h] = G^T [lambda_x~^{n+1}; lambda_y^{n+1}]
//                  per model (row blocks of G^T), lambda_h added into the
//                  adjoint Hz of the ring cells (each ring cell belongs to one
//                  port of one model, so the read-modify-write is unshared);
//   adj_stream   : the transpose of eq. (3) and eq. (5) with the gradient
//                  accumulation, streamed up the rows (one launch).
// The forward coefficients are rebuilt exactly as the step kernel builds
// them.
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "../../include/fdtd_rom.h"
#include "adjoint.hpp"
#include "device.hpp"

// Workspace of the reverse sweep that allocates nothing
// (fdtd_rom_adjoint_noalloc): every GPU the library runs on holds one copy,
// zero-initialised at load, until the process ends.  Host code never passes
// this name to a kernel or copy (on the host it is only a stand-in for the
// symbol); it uses the per-device address noalloc_scratch() returns.
static __device__ __align__(256) unsigned char scratch[fdtd::kNoAllocScratchBytes];

namespace fdtd {

int noalloc_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FDTD_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return fail(FDTD_EDEVICE, "device %d beyond the %d the scratch table holds", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FDTD_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return FDTD_OK;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) transpose_block(const T* __restrict__ g, T* __restrict__ gt, int ldg,
                                                         int nc) {
  const size_t n = (size_t)ldg * ldg;
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (size_t)gridDim.x * kBlock) {
    const int c = (int)(k / ldg), r = (int)(k - (size_t)c * ldg);
    gt[k] = (r < nc && c < nc) ? g[(size_t)r * ldg + c] : T(0);
  }
}

template <typename T>
hipError_t launch_transpose_block(const T* g, T* gt, int ldg, int nc, hipStream_t s) {
  const size_t n = (size_t)ldg * ldg;
  const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((n + kBlock - 1) / kBlock, 2048));
  hipLaunchKernelGGL((transpose_block<T>), dim3(nb), dim3(kBlock), 0, s, g, gt, ldg, nc);
  return hipGetLastError();
}

__global__ void rom_entry(RomDev* out, const RomDev* in, int64_t gt_off) {
  if (threadIdx.x == 0) {
    RomDev r = *in;
    r.g_off = -1;
    r.gt_off = gt_off;
    *out = r;
  }
}

hipError_t launch_rom_entry(RomDev* out, const RomDev* in, int64_t gt_off, hipStream_t s) {
  hipLaunchKernelGGL(rom_entry, dim3(1), dim3(kWave), 0, s, out, in, gt_off);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) probe_energy(const T* __restrict__ buf, int nprobes, int probe, int n,
                                                      double dt, double* out) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) {
    const double v = (double)buf[(size_t)k * nprobes + probe];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = dt * red[0];
}

template <typename T>
hipError_t launch_probe_energy(const T* buf, int nprobes, int probe, int n, double dt, double* out, hipStream_t s) {
  hipLaunchKernelGGL((probe_energy<T>), dim3(1), dim3(kBlock), 0, s, buf, nprobes, probe, n, dt, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock) zero_fill(uint4* p, size_t n) {
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (size_t)gridDim.x * kBlock)
    p[k] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 16 != 0 || ((uintptr_t)p) % 16 != 0) return hipErrorInvalidValue;
  const size_t n = bytes / 16;
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(zero_fill, dim3(nb), dim3(kBlock), 0, s, (uint4*)p, n);
  return hipGetLastError();
}

__global__ void rom_xstride(RomDev* out, const RomDev* in, int nroms, int64_t xstride) {
  for (int k = threadIdx.x; k < nroms; k += blockDim.x) {
    RomDev r = in[k];
    r.xstride = xstride;
    out[k] = r;
  }
}

hipError_t launch_rom_xstride(RomDev* out, const RomDev* in, int nroms, int64_t xstride, hipStream_t s) {
  if (nroms <= 0) return hipSuccess;
  hipLaunchKernelGGL(rom_xstride, dim3(1), dim3(kBlock), 0, s, out, in, nroms, xstride);
  return hipGetLastError();
}

// one workgroup per region
template <typename T>
__global__ void __launch_bounds__(kBlock) states_to_image(const T* __restrict__ src, T* __restrict__ dst,
                                                        const RomDev* __restrict__ roms, int par) {
  const RomDev r = roms[blockIdx.x];
  for (int a = threadIdx.x; a < r.q; a += kBlock) dst[r.x_off + a] = src[r.x_off + par * r.xstride + a];
}

template <typename T>
hipError_t launch_states_to_image(const T* src, T* dst, const RomDev* roms, int nroms, int par, hipStream_t s) {
  if (nroms <= 0) return hipSuccess;
  hipLaunchKernelGGL((states_to_image<T>), dim3(nroms), dim3(kBlock), 0, s, src, dst, roms, par);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) image_to_states(const T* __restrict__ src, T* __restrict__ dst,
                                                        const RomDev* __restrict__ roms, int par) {
  const RomDev r = roms[blockIdx.x];
  for (int a = threadIdx.x; a < r.q; a += kBlock) dst[r.x_off + par * r.xstride + a] = src[r.x_off + a];
}

template <typename T>
hipError_t launch_image_to_states(const T* src, T* dst, const RomDev* roms, int nroms, int par, hipStream_t s) {
  if (nroms <= 0) return hipSuccess;
  hipLaunchKernelGGL((image_to_states<T>), dim3(nroms), dim3(kBlock), 0, s, src, dst, roms, par);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) slots_to_probes(const T* __restrict__ slot0, size_t stride, size_t fe,
                                                        int len, int nprobes, const int* __restrict__ off,
                                                        const int* __restrict__ comp, T* __restrict__ buf, int m0) {
  const size_t n = (size_t)len * nprobes;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
    const size_t k = e / nprobes, t = e - k * nprobes;
    buf[((size_t)m0 + k) * nprobes + t] = slot0[k * stride + (size_t)comp[t] * fe + off[t]];
  }
}

template <typename T>
hipError_t launch_slots_to_probes(const T* slot0, size_t stride, size_t fe, int len, int nprobes, const int* off,
                                  const int* comp, T* buf, int m0, hipStream_t s) {
  const size_t n = (size_t)len * nprobes;
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL((slots_to_probes<T>), dim3(nb), dim3(kBlock), 0, s, slot0, stride, fe, len, nprobes, off, comp,
                     buf, m0);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kBlock) zero_padding(T* __restrict__ base, size_t count, int ny, int pitch, int nx) {
  const int w = pitch - nx;
  const size_t n = count * (size_t)ny * w;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
    const size_t row = e / w;  // row over all arrays
    base[row * pitch + nx + (e - row * w)] = T(0);
  }
}

template <typename T>
hipError_t launch_zero_padding(T* base, size_t count, int ny, int pitch, int nx, hipStream_t s) {
  const size_t n = count * (size_t)ny * (size_t)(pitch - nx);
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL((zero_padding<T>), dim3(nb), dim3(kBlock), 0, s, base, count, ny, pitch, nx);
  return hipGetLastError();
}

template hipError_t launch_zero_padding<float>(float*, size_t, int, int, int, hipStream_t);
template hipError_t launch_zero_padding<double>(double*, size_t, int, int, int, hipStream_t);
template hipError_t launch_image_to_states<float>(const float*, float*, const RomDev*, int, int, hipStream_t);
template hipError_t launch_image_to_states<double>(const double*, double*, const RomDev*, int, int, hipStream_t);
template hipError_t launch_slots_to_probes<float>(const float*, size_t, size_t, int, int, const int*, const int*,
                                                  float*, int, hipStream_t);
template hipError_t launch_slots_to_probes<double>(const double*, size_t, size_t, int, int, const int*, const int*,
                                                   double*, int, hipStream_t);
template hipError_t launch_states_to_image<float>(const float*, float*, const RomDev*, int, int, hipStream_t);
template hipError_t launch_states_to_image<double>(const double*, double*, const RomDev*, int, int, hipStream_t);
template hipError_t launch_transpose_block<float>(const float*, float*, int, int, hipStream_t);
template hipError_t launch_transpose_block<double>(const double*, double*, int, int, hipStream_t);
template hipError_t launch_probe_energy<float>(const float*, int, int, int, double, double*, hipStream_t);
template hipError_t launch_probe_energy<double>(const double*, int, int, int, double, double*, hipStream_t);

// mu of a cell outside the layers: its adjoint Hz plus the coupling's
// lambda_h (0 off the ring cells) and the objective term, then the E
// update's transposes of its south, north, west and east edges, in this
// order and uncontracted, so that the stream and the fused coupling blocks
// form the same value bit for bit
template <typename T>
__device__ __forceinline__ T mu_plain(T lh, T pend, T obj, bool aS, T cS, T lS, bool aN, T cN, T lN, bool aW, T cW,
                                      T lW, bool aE, T cE, T lE) {
#pragma clang fp contract(off)
  T mu = lh + pend;
  mu += obj;
  mu += aS ? cS * lS : T(0);
  mu -= aN ? cN * lN : T(0);
  mu -= aW ? cW * lW : T(0);
  mu += aE ? cE * lE : T(0);
  return mu;
}

template <typename T>
__device__ __forceinline__ void adj_coef(T s, T t, T k2, T& ca, T& cb, T& rcp) {
#pragma clang fp contract(off)
  rcp = T(1) / (s + t);
  ca = (s - t) * rcp;
  cb = k2 * rcp;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adj_coupling(const AdjParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* z = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  const RowBlock rb = p.blocks[blockIdx.x];
  const RomDev r = p.roms[rb.a];
  const T* lxin = p.lx_in + r.x_off;
  T* lxout = p.lx_out + r.x_off;
  const int* gi = p.idx + r.i_off;
  const int* si = gi + r.np;
  const int lane = tid & (kWave - 1);
  const int row0 = rb.b + (tid / kWave) * kRowsPerWave;
  const T* GT = p.mats + r.gt_off + (size_t)row0 * r.ldg;  // row k of G^T = column k of G
  T acc[kRowsPerWave];
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) acc[k] = T(0);
  auto stage = [&]() {
    for (int c = tid; c < r.ldg; c += kBlock) {
      T v = T(0);
      if (c < r.q) {
        v = lxin[c];
      } else if (c < r.q + r.np) {
        const int pp = c - r.q;
        v = (pp < r.n_ex ? p.lex_in : p.ley_in)[si[pp]];
      }
      z[c] = v;
    }
    lds_barrier();
  };
  lane_row_dots<T, kRowsPerWave>(GT, r.ldg, z, lane, acc, stage);
  if (p.dgt) {
    // dJ/dG^T row c += (input c of step n) x (adjoint of the outputs), FP64
    const int nc = r.q + r.np;
    double* dg = p.dgt + p.dg_off[rb.a];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int row = row0 + k;
      if (row >= nc) break;
      const double zin = (double)(row < r.q ? p.xn[r.x_off + row] : p.hz1[gi[row - r.q]]);
      double* d = dg + (size_t)row * r.ldg;
      for (int c = lane; c < nc; c += kWave) d[c] += zin * (double)z[c];
    }
  }
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k)
    for (int o = kWave / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, kWave);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int row = row0 + k;
      if (row < r.q)
        lxout[row] = acc[k];
      else if (row < r.q + r.np)
        p.lhz_in[gi[row - r.q]] += acc[k];
    }
  }
}

// dJ/da and dJ/db shares of one active edge (a, b the edge means of
// eps0*eps_r/dt and sigma/2): with s = a1+a2, t = b1+b2 and rcp = 1/(s+t)
// (the eq. (3) coefficients' own reciprocal), Ca = (s-t) rcp and
// Cb/d = 2 rcp/d, so dCa/da = 2b/(a+b)^2 = 4 rcp^2 t, dCa/db = -4 rcp^2 s,
// d(Cb/d)/da = d(Cb/d)/db = -4 rcp^2/d.  Weights: lam E^n for Ca and
// lam (Hz difference) for Cb/d; no division.
template <typename T>
__device__ __forceinline__ void edge_grad(T lam, T e_old, T dh, T s, T t, T rcp, T invd, T& ga, T& gb) {
  const T r2 = T(4) * rcp * rcp;
  const T dca = lam * e_old;
  const T u = lam * dh * invd;
  ga += r2 * (dca * t - u);
  gb += r2 * (-dca * s - u);
}

// One lane's column of row j for the reverse sweep.  With absorbing layers
// also the adjoints of the four auxiliary fields the column owns and the
// forward auxiliary fields at its Ex and Ey after the step.
template <typename T>
struct AdjRow {
  T a, b, h;      // material (a < 0 inside regions, 0 in padding), forward Hz^{n+1/2}
  T lx, e;        // adjoint and forward value of the row's south Ex
  T lh, ly, ey;   // adjoint Hz, adjoint and forward value of the west Ey
  T lpx, lpy;     // adjoints of the cell's psi (d/dx of Ey, d/dy of Ex)
  T lpe, lpw;     // adjoints of psi at the south Ex and at the west Ey
  T pe, pw;       // forward psi at the south Ex and the west Ey, after the step
};

// Loads are unconditional from a valid offset (`ob` when `ok`, else cell
// (0,0)) and the values of lanes without data are selected to zero: no
// lane-divergent branches.
template <typename T, bool PML>
__device__ __forceinline__ AdjRow<T> adj_load(const AdjParams<T>& p, uint32_t ob, bool ok) {
  const uint32_t o = ok ? ob : 0u;
  AdjRow<T> r{};
  if (p.midx) {
    const MatPair<T> m = p.mt[ld(p.mi, o / (uint32_t)(sizeof(T) / sizeof(uint16_t)))];
    r.a = m.a;
    r.b = m.b;
  } else {
    r.a = ld(p.al, o);
    r.b = ld(p.be, o);
  }
  r.h = ld(p.hz1, o);
  r.lx = ld(p.lex_in, o);
  r.e = ld(p.ex0, o);
  r.lh = ld(p.lhz_in, o);
  r.ly = ld(p.ley_in, o);
  r.ey = ld(p.ey0, o);
  if constexpr (PML) {
    r.lpx = ld(p.lps_in[0], o);
    r.lpy = ld(p.lps_in[1], o);
    r.lpe = ld(p.lps_in[2], o);
    r.lpw = ld(p.lps_in[3], o);
    r.pe = ld(p.pex1, o);
    r.pw = ld(p.pey1, o);
  }
  if (!ok) r = AdjRow<T>{};
  return r;
}

// Stretched-derivative profiles at one column (x) or row (y): 1/kappa, b, a
// at the E sample and at the Hz sample; the identity (1, 1, 0) outside the
// layers.
template <typename T>
struct Prof {
  T ik_e, b_e, a_e, ik_h, b_h, a_h;
};

template <typename T>
__device__ __forceinline__ Prof<T> prof_at(const T* pr, int S, int k) {
  return Prof<T>{pr[k], pr[S + k], pr[2 * S + k], pr[3 * S + k], pr[4 * S + k], pr[5 * S + k]};
}

constexpr int kAdjOwned = kWave - 3;  // columns a reverse-sweep wave owns

// Transposed eq. (3) + eq. (5) and the coefficient gradients, streamed up
// the rows like the forward stencil.  A wave covers 64 lanes = columns
// iw-2 .. iw+61 (iw = 61 * bx, tile column bx).  Lanes 2..62 own their column; lane 1
// only supplies mu of column iw-1 (its own west neighbour comes from lane
// 0), lanes 0 and 63 only supply data, so no lane loads anything outside
// its own column.  A segment of SEG rows recomputes mu of the row below it;
// rows j+1 and j+2 are in flight while row j is computed (the loop is
// unrolled: the row pipeline is register renaming).  Per row:
//   mu      = M (lambda_Hz' + objective + Cb_s lx_s - Cb_n lx_n - Cb_w ly_w
//             + Cb_e ly_e) over the cell's active edges;
//   lambda_Ex(j)  = chdy (mu(j-1) - mu(j)) + Ca lx  (Ca term on active edges);
//   lambda_Ey(i)  = chdx (mu(i) - mu(i-1)) + Ca ly;
//   gradients: every lane forms its west and east edges' shares; a south
//   edge is formed once and credited to both of its cells (a cell's total is
//   stored after its north edge, the next row's south edge, is known).
// Horizontal neighbours move between lanes with DPP whole-wave shifts.
//
// PML: the absorbing-layer form.  An E update E' = Ca E + Cb (dH/kappa +
// psi'), psi' = b psi + a dH hands its Hz difference the adjoint
//   v = Cb lam_E / kappa + a t,  t = lam_psi + Cb lam_E  (Ey: Cb -> -Cb),
// which replaces Cb lam_E in mu, and leaves b t to psi (edges the step
// updates; others keep their adjoint).  The Hz update hands
//   ldE = chdy mu / kappa_y + a_y (lam_psiy + chdy mu)  (x: chdx -> -chdx)
// to its E difference and b (lam_psi +- chd mu) to its own psi; the E
// adjoints become ldE(below) - ldE(own), and the Cb weights take the
// stretched difference dH/kappa + psi'.
template <typename T, int SEG, bool PML>
__device__ __forceinline__ void adj_rows(const AdjParams<T>& p, int bx, int by) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int iw = bx * kAdjOwned;
  const int ic = iw - 2 + lane;
  const int j0 = (by * (kBlock / kWave) + wv) * SEG;
  const int j1 = min(j0 + SEG, p.ny);
  const int js = j0 > 0 ? j0 - 1 : 0;
  const int nx = p.nx, ny = p.ny;
  constexpr uint32_t ts = sizeof(T);
  const uint32_t row_b = (uint32_t)p.pitch * ts;
  const bool in = ic >= 0 && ic < nx;
  const bool own = in && lane >= 2 && lane <= kWave - 2;
  const T chdy = p.chdy, chdx = p.chdx, k2dy = p.k2dy, k2dx = p.k2dx;
  const T idx = T(1.0 / p.dx), idy = T(1.0 / p.dy);  // reciprocal lengths
  const T fa = T(p.fa);
  // byte offset of (ic, js); only dereferenced where `in`
  uint32_t ob = ((uint32_t)js * (uint32_t)p.pitch + (uint32_t)ic) * ts;
  const uint32_t obj_b = (uint32_t)(p.obj_off * ts);
  // x profiles of this column and the east edge's (column ic+1)
  Prof<T> px{T(1), T(1), T(0), T(1), T(1), T(0)};
  T ikxE = T(1), axE = T(0);
  if constexpr (PML) {
    px = prof_at(p.px, p.px_stride, in ? ic : 0);
    ikxE = lane_next(px.ik_e);
    axE = lane_next(px.a_e);
  }

  AdjRow<T> prv = adj_load<T, PML>(p, ob - row_b, in && js >= 1);
  AdjRow<T> cur = adj_load<T, PML>(p, ob, in);
  AdjRow<T> nxt = adj_load<T, PML>(p, ob + row_b, in && js + 1 < ny);
  T mu_p = T(0), ld_p = T(0);
  T gpa = T(0), gpb = T(0);             // previous row's cell: dJ/da, dJ/db of all edges but its north
  T acc_e = T(0), acc_s = T(0);         // its accumulators, read one row ahead
  T cas = T(0), cbs = T(0), rs = T(0);  // current row's south edge
  adj_coef(cur.a + prv.a, cur.b + prv.b, k2dy, cas, cbs, rs);
#pragma unroll
  for (int it = 0; it <= SEG; ++it) {
    const int j = js + it;
    if (j >= j1) break;
    const bool up = j + 1 < ny;
    // row j+2 in flight (needed as the north row of the next iteration)
    const bool up2 = j + 2 < ny && j + 1 < j1;
    const AdjRow<T> nn = adj_load<T, PML>(p, ob + 2 * row_b, in && up2);
    // this row's accumulators (this wave is their only writer), stored next row
    const bool acc_row = j >= j0 && own;
    T nacc_e = ld(p.ga_e, acc_row ? ob : 0u);
    T nacc_s = ld(p.ga_s, acc_row ? ob : 0u);
    // horizontal neighbours
    const T aw = lane_prev(cur.a), bw = lane_prev(cur.b), hw = lane_prev(cur.h);
    const T ae = lane_next(cur.a), be_ = lane_next(cur.b), he = lane_next(cur.h);
    const T lye = lane_next(cur.ly), eye = lane_next(cur.ey);
    T caw, cbw, rw, cae, cbe, re, can, cbn, rn;
    adj_coef(cur.a + aw, cur.b + bw, k2dx, caw, cbw, rw);       // west edge (ic-1 | ic)
    adj_coef(ae + cur.a, be_ + cur.b, k2dx, cae, cbe, re);      // east edge (ic | ic+1)
    adj_coef(nxt.a + cur.a, nxt.b + cur.b, k2dy, can, cbn, rn); // north edge (j | j+1)
    const bool act = cur.a > T(0);
    const bool actS = j >= 1 && act && prv.a > T(0);
    const bool actN = up && act && nxt.a > T(0);
    const bool actW = ic >= 1 && act && aw > T(0);
    const bool actE = ic + 1 < nx && act && ae > T(0);
    // fused form: eq. (23)'s lambda_h of this step at a ring cell (an
    // active cell with a side on a region cell)
    T pend = T(0);
    if (p.pend_in) {
      const bool ring = act && (prv.a < T(0) || nxt.a < T(0) || aw < T(0) || ae < T(0));
      pend = ring ? ld(p.pend_in, ob) : T(0);
    }
    const T obj = (in && ob == obj_b) ? p.obj_coef * cur.h : T(0);
    T mu = cur.lh + pend;
    // y profiles of this row and of its north edge (wave-uniform)
    Prof<T> py{T(1), T(1), T(0), T(1), T(1), T(0)};
    T ikyN = T(1), ayN = T(0);
    T tS = T(0), tW = T(0), pwE = T(0);
    if constexpr (PML) {
      py = prof_at(p.py, p.py_stride, j);
      ikyN = p.py[j + 1];
      ayN = p.py[2 * p.py_stride + j + 1];
      const T lpwE = lane_next(cur.lpw);
      pwE = lane_next(cur.pw);
      tS = cur.lpe + cbs * cur.lx;
      tW = cur.lpw - cbw * cur.ly;
      const T tN = nxt.lpe + cbn * nxt.lx;
      const T tE = lpwE - cbe * lye;
      mu += obj;
      mu += actS ? cbs * py.ik_e * cur.lx + py.a_e * tS : T(0);
      mu -= actN ? cbn * ikyN * nxt.lx + ayN * tN : T(0);
      mu += actW ? -cbw * px.ik_e * cur.ly + px.a_e * tW : T(0);
      mu -= actE ? -cbe * ikxE * lye + axE * tE : T(0);
    } else {
      mu = mu_plain(cur.lh, pend, obj, actS, cbs, cur.lx, actN, cbn, nxt.lx, actW, cbw, cur.ly, actE, cbe, lye);
    }
    mu = act ? mu : T(0);
    // adjoints handed to the E differences of the Hz update (layers)
    T ldx = T(0), ldy = T(0), thx = T(0), thy = T(0);
    if constexpr (PML) {
      thy = cur.lpy + chdy * mu;
      thx = cur.lpx - chdx * mu;
      ldx = chdy * py.ik_h * mu + py.a_h * thy;
      ldy = -chdx * px.ik_h * mu + px.a_h * thx;
    }
    // west neighbour's value (all lanes take part in the shift)
    T mu_w = T(0), ldy_w = T(0);
    if constexpr (PML)
      ldy_w = lane_prev(ldy);
    else
      mu_w = lane_prev(mu);
    // gradient shares of the south, west and east edges; Cb weights the
    // (stretched) Hz difference
    T dhs = cur.h - prv.h, dhw = -(cur.h - hw), dhe = -(he - cur.h);
    if constexpr (PML) {
      dhs = py.ik_e * (cur.h - prv.h) + cur.pe;
      dhw = -(px.ik_e * (cur.h - hw) + cur.pw);
      dhe = -(ikxE * (he - cur.h) + pwE);
    }
    T gas = T(0), gbs = T(0), gaw = T(0), gbw = T(0), gae = T(0), gbe = T(0);
    edge_grad(cur.lx, cur.e, dhs, cur.a + prv.a, cur.b + prv.b, rs, idy, gas, gbs);
    edge_grad(cur.ly, cur.ey, dhw, cur.a + aw, cur.b + bw, rw, idx, gaw, gbw);
    edge_grad(lye, eye, dhe, ae + cur.a, be_ + cur.b, re, idx, gae, gbe);
    gas = actS ? gas : T(0);
    gbs = actS ? gbs : T(0);
    gaw = actW ? gaw : T(0);
    gbw = actW ? gbw : T(0);
    gae = actE ? gae : T(0);
    gbe = actE ? gbe : T(0);
    if (acc_row) {
      T lxo, lyo;
      if constexpr (PML) {
        lxo = (ld_p - ldx) + (actS ? cas * cur.lx : T(0));
        lyo = (ldy_w - ldy) + (actW ? caw * cur.ly : T(0));
        st(p.lps_out[0], ob, px.b_h * thx);
        st(p.lps_out[1], ob, py.b_h * thy);
        st(p.lps_out[2], ob, actS ? py.b_e * tS : cur.lpe);
        st(p.lps_out[3], ob, actW ? px.b_e * tW : cur.lpw);
      } else {
        lxo = chdy * (mu_p - mu) + (actS ? cas * cur.lx : T(0));
        lyo = chdx * (mu - mu_w) + (actW ? caw * cur.ly : T(0));
      }
      st(p.lhz_out, ob, mu);
      st(p.lex_out, ob, j >= 1 ? lxo : T(0));
      st(p.ley_out, ob, ic >= 1 ? lyo : T(0));
      // the previous row's cell is complete with its north edge (= this row's south)
      if (j - 1 >= j0) {
        st(p.ga_e, ob - row_b, acc_e + fa * (gpa + gas));
        st(p.ga_s, ob - row_b, acc_s + T(0.25) * (gpb + gbs));
      }
    }
    gpa = gas + gaw + gae;
    gpb = gbs + gbw + gbe;
    acc_e = nacc_e;
    acc_s = nacc_s;
    mu_p = mu;
    ld_p = ldx;
    prv = cur;
    cur = nxt;
    nxt = nn;
    cas = can;
    cbs = cbn;
    rs = rn;
    ob += row_b;
  }
  // last row's cell: add its north edge (the south edge of row j1)
  if (own && j1 - 1 >= j0) {
    const uint32_t oc = ob - row_b;
    T gna = T(0), gnb = T(0);
    if (j1 < ny && prv.a > T(0) && cur.a > T(0)) {
      T dhn = cur.h - prv.h;
      if constexpr (PML) dhn = p.py[j1] * (cur.h - prv.h) + cur.pe;
      edge_grad(cur.lx, cur.e, dhn, cur.a + prv.a, cur.b + prv.b, rs, idy, gna, gnb);
    }
    st(p.ga_e, oc, acc_e + fa * (gpa + gna));
    st(p.ga_s, oc, acc_s + T(0.25) * (gpb + gnb));
  }
}

// A wave takes the absorbing-layer form only when the profiles it reads
// (columns iw-2 .. iw+61, rows js .. j1) reach into a layer; kernels built
// for problems without layers contain the plain form only.  The adjoints
// of the auxiliary fields are written by layer waves alone: outside the
// layers every a is zero, so the entries other waves own stay zero and
// are never weighted.
template <typename T, int SEG, bool Layers>
__device__ __forceinline__ void adj_tile(const AdjParams<T>& p, int bx, int by) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int j0 = (by * (kBlock / kWave) + wv) * SEG;
  if (j0 >= p.ny) return;
  if constexpr (!Layers) {
    adj_rows<T, SEG, false>(p, bx, by);
  } else {
    const int iw = bx * kAdjOwned;
    const int js = j0 > 0 ? j0 - 1 : 0;
    const int j1 = min(j0 + SEG, p.ny);
    const bool layer = (p.pml_xlo > 0 && iw - 2 < p.pml_xlo) ||
                       (p.pml_xhi > 0 && iw + kWave - 3 >= p.nx - p.pml_xhi) ||
                       (p.pml_ylo > 0 && js < p.pml_ylo) || (p.pml_yhi > 0 && j1 >= p.ny - p.pml_yhi);
    if (layer)
      adj_rows<T, SEG, true>(p, bx, by);
    else
      adj_rows<T, SEG, false>(p, bx, by);
  }
}

// Stream workgroup s of n8 (a multiple of 8) -> tile index: each of the 8
// XCDs (workgroup s runs on XCD s % 8 when the stream part starts at a
// multiple of 8) takes a contiguous run of tiles, so vertically and
// laterally neighbouring tiles, which read each other's halo rows and
// lines, mostly share an L2.
__device__ __forceinline__ int adj_xcd_tile(int s, int n8) { return (s & 7) * (n8 >> 3) + (s >> 3); }

template <typename T, int SEG, bool Layers>
__global__ void __launch_bounds__(kBlock) adj_stream(const AdjParams<T> p, int gx, int ntiles) {
  const int t = adj_xcd_tile(blockIdx.x, (int)gridDim.x);
  if (t >= ntiles) return;
  adj_tile<T, SEG, Layers>(p, t % gx, t / gx);
}

// mu of an active cell at offset `off` as adj_rows forms it (no absorbing
// layer reaches a ring cell): the adjoint of its Hz^{n+1/2} after the
// coupling's and the E update's transposes, same terms in the same order
template <typename T>
__device__ __forceinline__ T ring_mu(const AdjParams<T>& p, int off) {
  const int P = p.pitch;
  const int j = off / P, i = off - j * P;
  const T a = p.al[off], b = p.be[off];
  if (!(a > T(0))) return T(0);
  T ca, cS = T(0), cN = T(0), cW = T(0), cE = T(0), rcp;
  const bool aS = j >= 1 && p.al[off - P] > T(0);          // south Ex(i, j)
  const bool aN = j + 1 < p.ny && p.al[off + P] > T(0);    // north Ex(i, j+1)
  const bool aW = i >= 1 && p.al[off - 1] > T(0);          // west Ey(i, j)
  const bool aE = i + 1 < p.nx && p.al[off + 1] > T(0);    // east Ey(i+1, j)
  if (aS) adj_coef(a + p.al[off - P], b + p.be[off - P], p.k2dy, ca, cS, rcp);
  if (aN) adj_coef(p.al[off + P] + a, p.be[off + P] + b, p.k2dy, ca, cN, rcp);
  if (aW) adj_coef(a + p.al[off - 1], b + p.be[off - 1], p.k2dx, ca, cW, rcp);
  if (aE) adj_coef(p.al[off + 1] + a, p.be[off + 1] + b, p.k2dx, ca, cE, rcp);
  const T obj = (off == p.obj_off) ? p.obj_coef * p.hz1[off] : T(0);
  return mu_plain(p.lhz_in[off], p.pend_in[off], obj, aS, cS, aS ? p.lex_in[off] : T(0), aN, cN,
                  aN ? p.lex_in[off + P] : T(0), aW, cW, aW ? p.ley_in[off] : T(0), aE, cE,
                  aE ? p.ley_in[off + 1] : T(0));
}

// Fused form, coupling block: eq. (23)'s transpose for step n-1.  Its input
// adjoint is [lambda_x^n; lambda_y^n]; lambda_y^n, the adjoint of E^n on the
// interface edges, is what the stream of step n writes there:
// +-chd * mu(ring cell) (S: chdy (mu - 0), N: chdy (0 - mu), W: chdx (0 - mu),
// E: chdx (mu - 0), the other side's cell lying in the region), formed here
// from step n's inputs with the stream's arithmetic.  lambda_h^{n-1} of each
// port goes to pend_out at its ring cell (each ring cell serves one port).
template <typename T>
__device__ __forceinline__ void coupling_fused_block(const AdjParams<T>& p, int blk, T* z) {
  const int tid = threadIdx.x;
  const RowBlock rb = p.blocks[blk];
  const RomDev r = p.roms[rb.a];
  const T* lxin = p.lx_in + r.x_off;
  T* lxout = p.lx_out + r.x_off;
  const int* gi = p.idx + r.i_off;
  const int lane = tid & (kWave - 1);
  const int row0 = rb.b + (tid / kWave) * kRowsPerWave;
  const T* GT = p.mats + r.gt_off + (size_t)row0 * r.ldg;
  const int ni = r.n_ex / 2;
  T acc[kRowsPerWave];
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) acc[k] = T(0);
  auto stage = [&]() {
    for (int c = tid; c < r.ldg; c += kBlock) {
      T v = T(0);
      if (c < r.q) {
        v = lxin[c];
      } else if (c < r.q + r.np) {
        const int k = c - r.q;
        const T mu = ring_mu(p, gi[k]);
        if (k < ni) v = p.chdy * (mu - T(0));
        else if (k < 2 * ni) v = p.chdy * (T(0) - mu);
        else if (k < r.n_ex + (r.np - r.n_ex) / 2) v = p.chdx * (T(0) - mu);
        else v = p.chdx * (mu - T(0));
      }
      z[c] = v;
    }
    lds_barrier();
  };
  lane_row_dots<T, kRowsPerWave>(GT, r.ldg, z, lane, acc, stage);
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k)
    for (int o = kWave / 2; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o, kWave);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int row = row0 + k;
      if (row < r.q)
        lxout[row] = acc[k];
      else if (row < r.q + r.np)
        p.pend_out[gi[row - r.q]] = acc[k];
    }
  }
}

// Fused reverse step: workgroups [0, ncoup) are coupling blocks of step n-1
// (first, so their chains start early), the rest, from the next multiple
// of 8, the stream of step n (workgroup ncoup8 + s takes tile
// adj_xcd_tile(s, n8), (t % gx, t / gx)).  The coupling blocks read
// only step n's inputs and write lx_out and pend_out, which no stream
// workgroup reads, so the two parts run side by side.
template <typename T, int SEG, bool Layers>
__global__ void __launch_bounds__(kBlock) adj_fused(const AdjParams<T> p, int ncoup, int gx, int ntiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int ncoup8 = (ncoup + 7) & ~7;
  if (b < ncoup8) {
    if (b < ncoup) coupling_fused_block(p, b, reinterpret_cast<T*>(smem));
    return;
  }
  const int t = adj_xcd_tile(b - ncoup8, (int)gridDim.x - ncoup8);
  if (t >= ntiles) return;
  adj_tile<T, SEG, Layers>(p, t % gx, t / gx);
}

template <typename T>
hipError_t launch_adjoint_step(const AdjParams<T>& p, size_t smem, hipStream_t s) {
  if (p.nblocks > 0) hipLaunchKernelGGL((adj_coupling<T>), dim3(p.nblocks), dim3(kBlock), smem, s, p);
  const int rows = (kBlock / kWave) * p.seg;
  const int gx = (p.nx + kAdjOwned - 1) / kAdjOwned, gy = (p.ny + rows - 1) / rows, nt = gx * gy;
  const dim3 g((unsigned)((nt + 7) & ~7));
  auto go = [&](auto layers) -> hipError_t {
    constexpr bool Ly = decltype(layers)::value;
    switch (p.seg) {
      case 2: hipLaunchKernelGGL((adj_stream<T, 2, Ly>), g, dim3(kBlock), 0, s, p, gx, nt); break;
      case 4: hipLaunchKernelGGL((adj_stream<T, 4, Ly>), g, dim3(kBlock), 0, s, p, gx, nt); break;
      case 8: hipLaunchKernelGGL((adj_stream<T, 8, Ly>), g, dim3(kBlock), 0, s, p, gx, nt); break;
      case 16: hipLaunchKernelGGL((adj_stream<T, 16, Ly>), g, dim3(kBlock), 0, s, p, gx, nt); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  return p.pml ? go(std::true_type{}) : go(std::false_type{});
}

template <typename T>
hipError_t launch_adjoint_fused(const AdjParams<T>& p, bool coupling, size_t smem, hipStream_t s) {
  const int rows = (kBlock / kWave) * p.seg;
  const int gx = (p.nx + kAdjOwned - 1) / kAdjOwned, gy = (p.ny + rows - 1) / rows;
  const int ncoup = coupling ? p.nblocks : 0, nt = gx * gy;
  const dim3 g((unsigned)(((ncoup + 7) & ~7) + ((nt + 7) & ~7)));
  const size_t lds = ncoup > 0 ? smem : 0;
  auto go = [&](auto layers) -> hipError_t {
    constexpr bool Ly = decltype(layers)::value;
    switch (p.seg) {
      case 2: hipLaunchKernelGGL((adj_fused<T, 2, Ly>), g, dim3(kBlock), lds, s, p, ncoup, gx, nt); break;
      case 4: hipLaunchKernelGGL((adj_fused<T, 4, Ly>), g, dim3(kBlock), lds, s, p, ncoup, gx, nt); break;
      case 8: hipLaunchKernelGGL((adj_fused<T, 8, Ly>), g, dim3(kBlock), lds, s, p, ncoup, gx, nt); break;
      case 16: hipLaunchKernelGGL((adj_fused<T, 16, Ly>), g, dim3(kBlock), lds, s, p, ncoup, gx, nt); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  return p.pml ? go(std::true_type{}) : go(std::false_type{});
}

__global__ void __launch_bounds__(kBlock) adj_flush(float* __restrict__ a, double* __restrict__ g, size_t n) {
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (size_t)gridDim.x * kBlock) {
    g[k] += (double)a[k];
    a[k] = 0.0f;
  }
}

hipError_t launch_adjoint_flush(float* a, double* g, size_t n, hipStream_t s) {
  const size_t nb = std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
  if (nb > 0) hipLaunchKernelGGL(adj_flush, dim3((unsigned)nb), dim3(kBlock), 0, s, a, g, n);
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjParams<float>&, size_t, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjParams<double>&, size_t, hipStream_t);
template hipError_t launch_adjoint_fused<float>(const AdjParams<float>&, bool, size_t, hipStream_t);
template hipError_t launch_adjoint_fused<double>(const AdjParams<double>&, bool, size_t, hipStream_t);

}  // namespace fdtd
