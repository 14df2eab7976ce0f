// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fdtd {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kMaxSrc = 4;         // sources applied inside the stencil kernel
constexpr int kMaxQ = 1024;        // reduced order handled by the coupling kernel
constexpr int kMaxPorts = 1024;    // ports per region
constexpr int kCtrlInts = 4;       // ctrl[0] = step, ctrl[1] = finished-block count

template <typename T>
struct Src {
  int comp, i0, i1, j0, j1;
  const T* incr;                   // device [max_steps]
};

// Device layout of the three field arrays: row-major with a common pitch,
//   Hz(i,j) at hz[j*pitch+i]   (j < ny)
//   Ex(i,j) at ex[j*pitch+i]   (j < ny; Ex(.,0) is the south wall, stored
//                                zero; Ex(.,ny) is the north wall, implicit)
//   Ey(i,j) at ey[j*pitch+i]   (i < nx; Ey(0,.) is the west wall, stored
//                                zero; Ey(nx,.) is the east wall, implicit)
// so every cell owns its Hz, its south Ex and its west Ey.
template <typename T>
struct StencilParams {
  const T* hz;
  const T* ex;
  const T* ey;
  T* hzo;
  T* exo;
  T* eyo;
  const T* al;       // per cell eps0*eps_r/dt; negative inside reduced regions
  const T* be;       // per cell sigma/2
  const int* ctrl;
  int nx, ny, pitch;
  int tiles_x, tiles_y, seg;
  T chdy, chdx;      // dt/(mu0 dy), dt/(mu0 dx)
  T k2dy, k2dx;      // 2/dy, 2/dx
  int nsrc;
  Src<T> src[kMaxSrc];
};

// One embedded model on the device.
struct RomDev {
  int q, np, n_ex;   // n_ex: ports [0, n_ex) are Ex (S, N), the rest Ey (W, E)
  int64_t m_off;     // [A~ | B~'] column-major q x (q+np), then C~ column-major np x q
  int64_t x_off;     // reduced state
  int64_t i_off;     // gather offsets [np] (Hz cells) then scatter offsets [np]
};

template <typename T>
struct CouplingParams {
  const RomDev* roms;
  int nroms;
  const T* mats;
  T* xs;
  const int* idx;
  const T* hz;       // step n+1 buffers
  T* ex;
  T* ey;
  int nprobes;
  const int* probe_off;
  const int* probe_comp;
  T* probe_buf;      // [max_steps][nprobes]
  int* ctrl;
  int nblocks;
};

// launchers (kernels.hip)
template <typename T>
hipError_t launch_stencil(const StencilParams<T>& p, int seg, hipStream_t s);
template <typename T>
hipError_t launch_coupling(const CouplingParams<T>& p, hipStream_t s);

}  // namespace fdtd
