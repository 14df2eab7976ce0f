// gfx950 kernels of the reverse (adjoint) sweep for the objective
//   J = dt * sum_n (Hz_p^{n+1/2})^2,
// the transpose of one forward step (eq. (23) coupling, eq. (3) E update,
// eq. (5) H update) applied in reverse order:
//   adj_coupling : [lambda_x~^n; lambda_h] = G^T [lambda_x~^{n+1}; lambda_y^{n+1}]
//                  per model (row blocks of G^T), lambda_h added into the
//                  adjoint Hz of the ring cells (each ring cell belongs to one
//                  port of one model, so the read-modify-write is unshared);
//   adj_mu       : per cell, mu = lambda_Hz' + objective term + the active
//                  edges' Cb-weighted lambda_E' (transpose of eq. (3) in Hz');
//                  lambda_Hz^n = mu on active cells; the cell's four edges add
//                  their dJ/deps_r and dJ/dsigma contributions (FP64);
//   adj_lame     : per edge, lambda_E^n = Ca lambda_E' on active edges plus
//                  the transpose of eq. (5) (differences of mu).
// The forward coefficients are rebuilt exactly as the step kernel builds
// them.  Thread per cell, 64 x 4 blocks, neighbour values from plain loads.
#include "adjoint.hpp"

namespace fdtd {

template <typename T>
__device__ __forceinline__ void adj_coef(T s, T t, T k2, T& ca, T& cb) {
#pragma clang fp contract(off)
  const T rcp = T(1) / (s + t);
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
  __syncthreads();
  const int lane = tid & (kWave - 1);
  const int row0 = rb.b + (tid / kWave) * kRowsPerWave;
  const T* GT = p.mats + r.gt_off + (size_t)row0 * r.ldg;  // row k of G^T = column k of G
  T acc[kRowsPerWave];
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) acc[k] = T(0);
  for (int c = lane; c < r.ldg; c += kWave) {
    const T zc = z[c];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) acc[k] += GT[(size_t)k * r.ldg + c] * zc;
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

// dJ/deps_r and dJ/dsigma of one active edge for the two cells sharing it:
// Ca = (a-b)/(a+b), Cb/d = 1/((a+b) d), a = mean eps/dt, b = mean sigma/2.
__device__ __forceinline__ void edge_grad(double lam, double e_old, double dh, double a1, double a2,
                                          double b1, double b2, double d, double fa, double& ge,
                                          double& gs) {
  const double a = 0.5 * (a1 + a2);
  const double b = 0.5 * (b1 + b2);
  const double s2 = (a + b) * (a + b);
  const double dca = lam * e_old;
  const double dcb = lam * dh;
  const double ga = dca * 2.0 * b / s2 - dcb / (s2 * d);
  const double gb = -dca * 2.0 * a / s2 - dcb / (s2 * d);
  ge += fa * ga;
  gs += 0.25 * gb;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adj_mu(const AdjParams<T> p) {
  const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
  const int j = blockIdx.y * (kBlock / kWave) + threadIdx.x / kWave;
  if (i >= p.nx || j >= p.ny) return;
  const size_t P = (size_t)p.pitch;
  const size_t o = (size_t)j * P + i;
  const T a = p.al[o];
  if (!(a > T(0))) {
    p.lhz_out[o] = T(0);
    return;
  }
  const T b = p.be[o];
  const T h = p.hz1[o];
  T mu = p.lhz_in[o];
  if ((int64_t)o == p.obj_off) mu += p.obj_coef * h;
  double ge = 0.0, gs = 0.0;
  const double fa = p.fa;
  // south Ex(i,j): cells (i,j-1), (i,j)
  if (j >= 1) {
    const T a2 = p.al[o - P];
    if (a2 > T(0)) {
      const T b2 = p.be[o - P];
      T ca, cb;
      adj_coef(a + a2, b + b2, p.k2dy, ca, cb);
      const T lam = p.lex_in[o];
      mu += cb * lam;
      edge_grad(lam, p.ex0[o], (double)h - (double)p.hz1[o - P], a, a2, b, b2, p.dy, fa, ge, gs);
    }
  }
  // north Ex(i,j+1): cells (i,j), (i,j+1)
  if (j + 1 < p.ny) {
    const T a2 = p.al[o + P];
    if (a2 > T(0)) {
      const T b2 = p.be[o + P];
      T ca, cb;
      adj_coef(a2 + a, b2 + b, p.k2dy, ca, cb);
      const T lam = p.lex_in[o + P];
      mu -= cb * lam;
      edge_grad(lam, p.ex0[o + P], (double)p.hz1[o + P] - (double)h, a, a2, b, b2, p.dy, fa, ge, gs);
    }
  }
  // west Ey(i,j): cells (i-1,j), (i,j)
  if (i >= 1) {
    const T a2 = p.al[o - 1];
    if (a2 > T(0)) {
      const T b2 = p.be[o - 1];
      T ca, cb;
      adj_coef(a + a2, b + b2, p.k2dx, ca, cb);
      const T lam = p.ley_in[o];
      mu -= cb * lam;
      edge_grad(lam, p.ey0[o], -((double)h - (double)p.hz1[o - 1]), a, a2, b, b2, p.dx, fa, ge, gs);
    }
  }
  // east Ey(i+1,j): cells (i,j), (i+1,j)
  if (i + 1 < p.nx) {
    const T a2 = p.al[o + 1];
    if (a2 > T(0)) {
      const T b2 = p.be[o + 1];
      T ca, cb;
      adj_coef(a2 + a, b2 + b, p.k2dx, ca, cb);
      const T lam = p.ley_in[o + 1];
      mu += cb * lam;
      edge_grad(lam, p.ey0[o + 1], -((double)p.hz1[o + 1] - (double)h), a, a2, b, b2, p.dx, fa, ge, gs);
    }
  }
  p.lhz_out[o] = mu;
  p.geps[o] += ge;
  p.gsig[o] += gs;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adj_lame(const AdjParams<T> p) {
  const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
  const int j = blockIdx.y * (kBlock / kWave) + threadIdx.x / kWave;
  if (i >= p.nx || j >= p.ny) return;
  const size_t P = (size_t)p.pitch;
  const size_t o = (size_t)j * P + i;
  const T a = p.al[o];
  const T b = p.be[o];
  const T mu = p.lhz_out[o];  // zero on inactive cells
  T lx = T(0), ly = T(0);
  if (j >= 1) {
    const T a2 = p.al[o - P];
    lx = p.chdy * (p.lhz_out[o - P] - mu);
    if (a > T(0) && a2 > T(0)) {
      T ca, cb;
      adj_coef(a + a2, b + p.be[o - P], p.k2dy, ca, cb);
      lx += ca * p.lex_in[o];
    }
  }
  if (i >= 1) {
    const T a2 = p.al[o - 1];
    ly = p.chdx * (mu - p.lhz_out[o - 1]);
    if (a > T(0) && a2 > T(0)) {
      T ca, cb;
      adj_coef(a + a2, b + p.be[o - 1], p.k2dx, ca, cb);
      ly += ca * p.ley_in[o];
    }
  }
  p.lex_out[o] = lx;
  p.ley_out[o] = ly;
}

template <typename T>
hipError_t launch_adjoint_step(const AdjParams<T>& p, size_t smem, hipStream_t s) {
  if (p.nblocks > 0) hipLaunchKernelGGL((adj_coupling<T>), dim3(p.nblocks), dim3(kBlock), smem, s, p);
  const dim3 g((p.nx + kWave - 1) / kWave, (p.ny + kBlock / kWave - 1) / (kBlock / kWave));
  hipLaunchKernelGGL((adj_mu<T>), g, dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL((adj_lame<T>), g, dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjParams<float>&, size_t, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjParams<double>&, size_t, hipStream_t);

}  // namespace fdtd
