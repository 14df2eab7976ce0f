// gfx950 kernels of the embedded-ROM FDTD time step.
//
//  yee_step  : fused coarse-grid leap-frog step (paper eqs. (5) then (3)):
//              Hz^{n-1/2} -> Hz^{n+1/2}, E^n -> E^{n+1}, with additive
//              sources; reads the step-n buffers, writes the step-(n+1)
//              buffers (ping-pong, so tiles can recompute their halo).
//  coupling  : per embedded model, eq. (23) in closed form: gather the coarse
//              Hz^{n+1/2} next to its ports, x~ <- A~ x~ + B~' h, y <- C~ x~,
//              scatter y^{n+1} into the interface edges; plus the probe
//              record and the device step counter.
//
// Stencil design (HBM-bound, one pass per step):
//   * a wave owns 64 adjacent columns and marches up a segment of SEG rows,
//     carrying Ex(i,j), Hz^{n+1/2}(i,j-1) and the material of row j-1 in
//     registers; the horizontal neighbours (Ey(i+1,j), Hz^{n+1/2}(i-1,j),
//     material of cell i-1) come from adjacent lanes by cross-lane moves,
//     lanes 0 and 63 fetch the one column outside the wave;
//   * each segment recomputes Hz^{n+1/2} of the row below it (one extra row
//     per SEG), so the whole step needs a single launch;
//   * per-edge coefficients are rebuilt from per-cell (a, b) =
//     (eps0*eps_r/dt, sigma/2): s = a1+a2, t = b1+b2, Ca = (s-t)/(s+t),
//     Cb/d = (2/d)/(s+t) - 32 algorithmic bytes per cell update instead of
//     the 40 a per-edge coefficient table would cost;
//   * cells inside a reduced region carry a < 0: their Hz stays zero and
//     the edges on and inside the region keep their value (the interface
//     edges are then written by the coupling kernel);
//   * workgroups are remapped so each of the 8 XCDs (own L2) takes a
//     contiguous band of tiles, keeping the halo rows within one L2.
#include "common.hpp"

namespace fdtd {

__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int xcd = bid & 7;
  const int local = bid >> 3;
  const int per = nblk >> 3;
  const int rem = nblk & 7;
  return (xcd < rem) ? xcd * (per + 1) + local
                     : rem * (per + 1) + (xcd - rem) * per + local;
}

template <typename T>
__device__ __forceinline__ void edge_coef(T s, T t, T k2, T& ca, T& cb) {
#pragma clang fp contract(off)
  const T rcp = T(1) / (s + t);
  ca = (s - t) * rcp;
  cb = k2 * rcp;
}

template <typename T>
__device__ __forceinline__ T src_sum(const StencilParams<T>& p, const T* sinc, int comp,
                                     int i, int j) {
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < kMaxSrc; ++s) {
    if (s < p.nsrc) {
      const Src<T>& S = p.src[s];
      if (S.comp == comp && i >= S.i0 && i < S.i1 && j >= S.j0 && j < S.j1) acc += sinc[s];
    }
  }
  return acc;
}

template <typename T, int SEG>
__global__ void __launch_bounds__(kBlock) yee_step(const StencilParams<T> p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % p.tiles_x;
  const int tyb = tile / p.tiles_x;
  const int i = tx * kWave + lane;
  const int j0 = (tyb * (kBlock / kWave) + wv) * SEG;
  if (j0 >= p.ny) return;  // uniform over the wave
  const int j1 = min(j0 + SEG, p.ny);
  const int nx = p.nx;
  const int ny = p.ny;
  const size_t P = (size_t)p.pitch;
  const bool in = i < nx;
  const bool has_left = (lane == 0) && (i >= 1);
  const bool has_right = (lane == kWave - 1) && (i + 1 < nx);
  const int n = p.ctrl[0];
  T sinc[kMaxSrc];
#pragma unroll
  for (int s = 0; s < kMaxSrc; ++s) sinc[s] = (s < p.nsrc) ? p.src[s].incr[n] : T(0);

  const int js = j0 > 0 ? j0 - 1 : 0;
  T ex_c = in ? p.ex[(size_t)js * P + i] : T(0);
  T exl_c = has_left ? p.ex[(size_t)js * P + i - 1] : T(0);
  T hn_prev = T(0), a_prev = T(0), b_prev = T(0);
  for (int j = js; j < j1; ++j) {
    const size_t o = (size_t)j * P + i;
    const bool up = (j + 1) < ny;
    T h = T(0), ex1 = T(0), ey0 = T(0), al = T(0), be = T(0);
    if (in) {
      h = p.hz[o];
      ex1 = up ? p.ex[o + P] : T(0);
      ey0 = p.ey[o];
      al = p.al[o];
      be = p.be[o];
    }
    T ey1 = __shfl_down(ey0, 1, kWave);
    if (lane == kWave - 1) ey1 = has_right ? p.ey[o + 1] : T(0);
    // eq. (5): Hz^{n+1/2}
    T hn = h + (p.chdy * (ex1 - ex_c) - p.chdx * (ey1 - ey0));
    hn += src_sum(p, sinc, 0, i, j);
    if (!(al > T(0))) hn = T(0);
    T hnl = __shfl_up(hn, 1, kWave);
    T all = __shfl_up(al, 1, kWave);
    T bel = __shfl_up(be, 1, kWave);
    if (lane == 0) {
      hnl = T(0);
      all = T(0);
      bel = T(0);
      if (has_left) {
        const T hl = p.hz[o - 1];
        const T exl1 = up ? p.ex[o - 1 + P] : T(0);
        const T eyl0 = p.ey[o - 1];
        all = p.al[o - 1];
        bel = p.be[o - 1];
        hnl = hl + (p.chdy * (exl1 - exl_c) - p.chdx * (ey0 - eyl0));
        hnl += src_sum(p, sinc, 0, i - 1, j);
        if (!(all > T(0))) hnl = T(0);
        exl_c = exl1;
      }
    }
    if (j >= j0 && in) {
      // eq. (3): Ex^{n+1}(i,j) between cells (i,j-1) and (i,j)
      T exn = ex_c;
      if (j >= 1 && al > T(0) && a_prev > T(0)) {
        T ca, cb;
        edge_coef(al + a_prev, be + b_prev, p.k2dy, ca, cb);
        exn = ca * ex_c + cb * (hn - hn_prev);
      }
      exn += src_sum(p, sinc, 1, i, j);
      // Ey^{n+1}(i,j) between cells (i-1,j) and (i,j)
      T eyn = ey0;
      if (i >= 1 && al > T(0) && all > T(0)) {
        T ca, cb;
        edge_coef(al + all, be + bel, p.k2dx, ca, cb);
        eyn = ca * ey0 - cb * (hn - hnl);
      }
      eyn += src_sum(p, sinc, 2, i, j);
      p.hzo[o] = hn;
      p.exo[o] = exn;
      p.eyo[o] = eyn;
    }
    hn_prev = hn;
    a_prev = al;
    b_prev = be;
    ex_c = ex1;
  }
}

// out = M v for column-major M (rows x cols), v and out in LDS.  Rows are
// split over threads, columns over `parts` thread groups, partial sums
// reduced through LDS.  Ends with a barrier.
template <typename T>
__device__ void block_matvec(const T* __restrict__ M, int rows, int cols, const T* v, T* out,
                             T* part) {
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < rows; r0 += kBlock) {
    const int R = min(rows - r0, kBlock);
    const int parts = kBlock / R;
    const int row = tid % R;
    const int pt = tid / R;
    T acc = T(0);
    if (pt < parts) {
      const int cper = (cols + parts - 1) / parts;
      const int c0 = pt * cper;
      const int c1 = min(cols, c0 + cper);
      const T* col = M + (size_t)c0 * rows + r0 + row;
      for (int c = c0; c < c1; ++c, col += rows) acc += *col * v[c];
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < R) {
      T s = T(0);
      for (int k = 0; k < parts; ++k) s += part[k * R + tid];
      out[r0 + tid] = s;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) coupling(const CouplingParams<T> p) {
  __shared__ T z[kMaxQ + kMaxPorts];
  __shared__ T xn[kMaxQ];
  __shared__ T part[kBlock];
  const int tid = threadIdx.x;
  const int n = p.ctrl[0];
  const int b = blockIdx.x;
  if (b < p.nroms) {
    const RomDev r = p.roms[b];
    const int q = r.q;
    const int np = r.np;
    const int nc = q + np;
    const T* M = p.mats + r.m_off;
    const T* C = M + (size_t)q * nc;
    T* x = p.xs + r.x_off;
    const int* gi = p.idx + r.i_off;
    const int* si = gi + np;
    for (int t = tid; t < nc; t += kBlock) z[t] = (t < q) ? x[t] : p.hz[gi[t - q]];
    __syncthreads();
    block_matvec(M, q, nc, z, xn, part);     // x~^{n+1} = A~ x~^n + B~' h
    for (int t = tid; t < q; t += kBlock) x[t] = xn[t];
    block_matvec(C, np, q, xn, z, part);     // y^{n+1} = C~ x~^{n+1}
    for (int t = tid; t < np; t += kBlock) {
      if (t < r.n_ex)
        p.ex[si[t]] = z[t];
      else
        p.ey[si[t]] = z[t];
    }
  } else {
    for (int t = tid; t < p.nprobes; t += kBlock) {
      const int c = p.probe_comp[t];
      const int o = p.probe_off[t];
      const T v = (c == 0) ? p.hz[o] : ((c == 1) ? p.ex[o] : p.ey[o]);
      p.probe_buf[(size_t)n * p.nprobes + t] = v;
    }
  }
  // every block has read ctrl[0]; the last one to finish advances the step
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const int prev = atomicAdd(&p.ctrl[1], 1);
    if (prev == p.nblocks - 1) {
      p.ctrl[1] = 0;
      p.ctrl[0] = n + 1;
      __threadfence();
    }
  }
}

template <typename T>
hipError_t launch_stencil(const StencilParams<T>& p, int seg, hipStream_t s) {
  const int rows = (kBlock / kWave) * seg;
  const int nblk = p.tiles_x * ((p.ny + rows - 1) / rows);
  const dim3 g(nblk), b(kBlock);
  switch (seg) {
    case 8: hipLaunchKernelGGL((yee_step<T, 8>), g, b, 0, s, p); break;
    case 16: hipLaunchKernelGGL((yee_step<T, 16>), g, b, 0, s, p); break;
    case 32: hipLaunchKernelGGL((yee_step<T, 32>), g, b, 0, s, p); break;
    case 64: hipLaunchKernelGGL((yee_step<T, 64>), g, b, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coupling(const CouplingParams<T>& p, hipStream_t s) {
  hipLaunchKernelGGL((coupling<T>), dim3(p.nblocks), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

template hipError_t launch_stencil<float>(const StencilParams<float>&, int, hipStream_t);
template hipError_t launch_stencil<double>(const StencilParams<double>&, int, hipStream_t);
template hipError_t launch_coupling<float>(const CouplingParams<float>&, hipStream_t);
template hipError_t launch_coupling<double>(const CouplingParams<double>&, hipStream_t);

}  // namespace fdtd
