// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fdtd {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kMaxSrc = 4;         // sources applied inside the stencil kernel
constexpr int kMaxQ = 16384;       // model order handled by the coupling kernels (also bounded by kMaxStageBytes)
constexpr int kMaxStageBytes = 65536;  // LDS of a coupling workgroup's staged [x~; h] (padded q + np elements)
constexpr int kMaxPorts = 1024;    // ports per region
constexpr int kCtrlInts = 4;       // ctrl[0] = step, ctrl[2] = non-finite flag (finite_check_kernel)

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
// so every cell owns its Hz, its south Ex and its west Ey.  Two such sets
// ping-pong: the state after n steps (E^n, Hz^{n-1/2}) lives in set n & 1.

// One embedded model on the device.  Its update is eq. (23) written as one
// matrix on z = [x~^n; h^{n+1/2}]:
//   [x~^{n+1}; y^{n+1}] = G z,  G = [[A~, B~'], [C~ A~, C~ B~']],
// rows padded to a multiple of kRowsPerBlock, row stride ldg (multiple of 64).
struct RomDev {
  int q, np, n_ex;   // n_ex: ports [0, n_ex) are Ex (S, N), the rest Ey (W, E)
  int ldg;           // padded row length of G (>= q + np)
  int64_t g_off;     // G, row-major
  int64_t x_off;     // reduced state, two buffers of xstride (step parity)
  int64_t xstride;
  int64_t i_off;     // gather offsets [np] (Hz cells) then scatter offsets [np]
  int64_t gt_off;    // G column-major (leading dimension ldg) for the shared-model GEMM, -1 if none
};

constexpr int kRowsPerWave = 4;
constexpr int kRowsPerBlock = kRowsPerWave * (kBlock / kWave);
constexpr int kGemmCopies = 16;    // copies (columns) per shared-model GEMM block
constexpr int kGemmRowsPerBlock = 64;  // output rows per GEMM block: one 16-row MFMA tile per wave
constexpr int kMaxGemmM = 512;     // q + np handled by the GEMM blocks
constexpr int kMinGemmCopies = 8;  // shared groups at least this large use the GEMM

// One coupling workgroup.  kind 0: rows [row0, row0 + kRowsPerBlock) of
// region `a`'s update matrix (GEMV).  kind 1: FP32 MFMA GEMM of one shared
// model for up to kGemmCopies regions listed at copies[b .. b + c), output
// 16-row tiles a .. a+3 (one per wave).
struct RowBlock {
  int kind;
  int a;
  int b;
  int c;
};

// Everything one leap-frog step needs.  One launch advances every tile of
// the coarse grid and every embedded model from step n to n+1, where
// n = ctrl[0] + step_off (ctrl[0] is advanced by a tick launch after each
// batch of steps, so a captured batch can be replayed).
// One entry of the material table: a = eps0*eps_r/dt (negative inside
// reduced regions), b = sigma/2 - the two per-cell numbers of eq. (3).
template <typename T>
struct alignas(2 * sizeof(T)) MatPair {
  T a, b;
};
constexpr int kMaxMaterials = 65536;

template <typename T>
struct StepParams {
  T* f[2][3];        // field sets [parity][Hz, Ex, Ey]
  const T* al;       // per cell eps0*eps_r/dt; negative inside reduced regions
  const T* be;       // per cell sigma/2
  // the same material as a 16-bit index per cell into a table of (a, b)
  // pairs, when the problem has at most kMaxMaterials distinct pairs
  const uint16_t* mi;
  const MatPair<T>* mt;
  int midx;          // 1: mi/mt hold the material (the stencil may use them)
  int* ctrl;
  int step_off;
  int nx, ny, pitch;
  int tiles_x, nst_blocks;
  int seg;           // rows per stencil wave (8, 16, 32) of this tiling
  T chdy, chdx;      // dt/(mu0 dy), dt/(mu0 dx)
  T k2dy, k2dx;      // 2/dy, 2/dx
  int nsrc;
  Src<T> src[kMaxSrc];
  // embedded models
  const RomDev* roms;
  const RowBlock* blocks;
  const int* copies; // region lists of the GEMM blocks
  int nrowblocks;    // real coupling blocks
  int ncoup_blocks;  // coupling blocks padded to a multiple of 8 (XCD alignment)
  const T* mats;
  T* xs;
  const int* idx;
  // probes
  int nprobes;
  const int* probe_off;
  const int* probe_comp;
  T* probe_buf;      // [max_steps][nprobes]
  // absorbing layers (pml == 0: none).  Profiles of the stretched
  // derivatives: px[k * px_stride + i] for k = 0..5 = (1/kappa, b, a) at the
  // Ey sample x = i dx, then at the Hz sample x = (i+1/2) dx; py likewise
  // along y (Ex at y = j dy, Hz at (j+1/2) dy).  Auxiliary fields (pitch
  // layout): the two at Hz by step parity, the ones at Ex and Ey in place.
  int pml;
  int pml_xlo, pml_xhi, pml_ylo, pml_yhi;
  int px_stride, py_stride;
  const T* px;
  const T* py;
  T* psi_h[2][2];    // [parity][d/dx of Ey, d/dy of Ex]
  T* psi_ex;         // d/dy of Hz at Ex
  T* psi_ey;         // d/dx of Hz at Ey
  // two-step launches (no absorbing layers): tiles of kOwned2 columns x
  // 4 SEG rows; role2[tile] 0 = far (two steps into f2), 1 = near a region
  // or a source (two steps into f2 except the band around each region, and
  // step n+1 of its cells into the step-(n+1) set); near_list: the n_near
  // near tiles, run as pieces of near_rows-row waves; far tiles [0,
  // far_split) run in the first launch, the rest in the second; n_band:
  // regions whose band the second launch advances.  In the second launch's
  // parameters f2 is the pair's step-n set.
  T* f2[3];
  int tiles_x2, nst2_blocks, n_near, n_band, near_rows, far_split;
  const uint8_t* role2;
  const int* near_list;
  // per cell (pitch layout): non-zero where a near tile stores step n+1 -
  // the cells the second launch reads from the step-(n+1) set (the band
  // blocks and the coupling's ring gathers: x in [i-1, i+2], y in [j-1, j+2]
  // around each ring cell (i, j)); nothing else reads that set
  const uint8_t* st1m;
};

constexpr int kOwned2 = kWave - 4;  // columns a two-step wave owns (lanes 2..61)
constexpr int kBandSplit = 4;       // workgroups per region's band in the second launch of a pair

// One workgroup of the batched step launch: instance `inst`, role `kind`
// (0 coupling block idx of that instance, 1 stencil tile idx, 2 probe
// block, 3 idle padding that keeps every instance's tile range aligned to
// the 8 XCDs).
struct BatchRef {
  int inst;
  int kind;
  int idx;
  int pad;
};

// Record a failure message for fdtd_rom_last_error() and return code.
int fail(int code, const char* fmt, ...);

// launchers (kernels.hip)
template <typename T>
hipError_t launch_step(const StepParams<T>& p, int seg, size_t smem, hipStream_t s);
// the pair of launches that advances steps n, n+1 (n = ctrl[0] + step_off)
template <typename T>
hipError_t launch_step2(const StepParams<T>& a, const StepParams<T>& b, int seg, size_t smem, hipStream_t s);
template <typename T>
hipError_t launch_probe_flush(const StepParams<T>& p, hipStream_t s);
hipError_t launch_tick(int* ctrl, int k, hipStream_t s);
// Sets *flag = 1 if any of the n elements at f is not finite (n a multiple
// of 16 bytes of elements, f 16-byte aligned); the flag is not cleared.
template <typename T>
hipError_t launch_finite_check(const T* f, size_t n, int* flag, hipStream_t s);
template <typename T>
hipError_t launch_energy(const T* hz, const T* ex, const T* ey, const T* al, int nx, int ny, int pitch,
                         double ch, double half_area, double dx, double dy, double* part, hipStream_t s);
inline int energy_blocks(int nx, int ny) {
  return ((nx + kWave - 1) / kWave) * ((ny + kBlock / kWave - 1) / (kBlock / kWave));
}
template <typename T>
hipError_t launch_batch_step(const StepParams<T>* descs, const BatchRef* table, int nblocks,
                             const int* ctrl, int step_off, size_t smem, bool layers, bool midx,
                             hipStream_t s);
// the pair of batched launches advancing steps n, n+1 of every instance
template <typename T>
hipError_t launch_batch_step2(const StepParams<T>* da, const BatchRef* ta, int na, const StepParams<T>* db,
                              const BatchRef* tb, int nb, const int* ctrl, int step_off, size_t smem, bool midx,
                              hipStream_t s);
template <typename T>
hipError_t launch_batch_probe_flush(const StepParams<T>* descs, int ninst, const int* ctrl,
                                    int step_off, hipStream_t s);

}  // namespace fdtd
