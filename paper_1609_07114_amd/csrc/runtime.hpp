// Internal state of a simulation handle, shared by the forward runtime
// (runtime.cpp) and the reverse sweep (adjoint_rt.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/fdtd_rom.h"
#include "common.hpp"

namespace fdtd {

inline constexpr double kC0 = FDTD_C0;
inline constexpr double kMu0 = FDTD_MU0;
inline const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte offsets of every array in the caller's device workspace.
struct Layout {
  int pitch = 0;
  size_t tsize = 0;
  size_t field_elems = 0;
  size_t off_ctrl = 0, off_fields = 0, off_al = 0, off_be = 0, off_src = 0;
  size_t off_pbuf = 0, off_poff = 0, off_pcomp = 0, off_roms = 0, off_mats = 0;
  size_t off_xs = 0, off_idx = 0, off_energy = 0, total = 0;
  size_t off_midx = 0, off_mtab = 0;  // 16-bit material index per cell; (a, b) table
  bool pml = false;                 // absorbing layers present
  int px_stride = 0, py_stride = 0; // profile row lengths (x: columns, y: rows)
  size_t off_prof = 0, off_psi = 0; // profiles [6][px] + [6][py]; 6 auxiliary fields
  // two-step launches (grids without layers): the step-(n+1) field set the
  // pair writes near regions, tile roles, near-tile list, near-probe flags
  bool tb_ok = false;
  int max_tiles2 = 0;
  size_t off_fc = 0, off_role2 = 0, off_near = 0, off_st1m = 0;
  size_t mats_elems = 0, xs_elems = 0, idx_elems = 0;
  int nrowblocks = 0;        // all-GEMV coupling list
  int nblocks_mixed = 0;     // GEMM for eligible shared groups + GEMV for the rest
  size_t off_blocks = 0, off_blocks_mixed = 0, off_copies = 0;
  std::vector<char> slot_gemm;     // slot uses the MFMA GEMM path
  std::vector<size_t> slot_gt_off; // element offset of the column-major copy
  std::vector<int> slot_members;   // regions per slot
  size_t ncopies = 0;
  size_t smem_gemv = 0, smem_mixed = 0;
  std::vector<int> slot_of_rom;     // matrix slot per region
  std::vector<int> slot_rep;        // representative region per slot
  std::vector<size_t> slot_off;     // element offset of each slot in the pool
  std::vector<size_t> x_off, i_off; // per region
};

inline int ports_of(const fdtd_rom& r) { return 2 * (r.ni + r.nj); }

// eq. (23) closed form of one region, FP64, row-major.
struct RomHost {
  int i0, j0, ni, nj, q, np, slot;
  std::vector<double> A, B, C;  // closed form, row-major
  std::vector<double> R;        // R~ (energy diagnostic)
  std::vector<double> F;        // F~ (gradients through the models)
  std::vector<double> cp, cm, sc;  // eq. (13) half cells C+, C- and Sc per port
};

}  // namespace fdtd

struct fdtd_rom_sim {
  int dtype = FDTD_F32;
  int nx = 0, ny = 0, pitch = 0;
  double dx = 0, dy = 0, dt = 0;
  int max_steps = 0, steps = 0, nprobes = 0, nsrc = 0, nroms = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  fdtd::Layout L;
  int seg = 16;
  int nmat = 0;           // material table entries (0: more distinct pairs than the table holds)
  size_t smem = 0;        // dynamic LDS of the step kernel
  bool shared_gemm = true;
  std::vector<fdtd::RomHost> roms;
  std::vector<fdtd_probe> probes;
  std::vector<unsigned char> pec;    // PEC cells [ny*nx] (empty: none)
  fdtd::StepParams<float> sp_f;
  fdtd::StepParams<double> sp_d;
  int graph_batch = 0;               // > 0: replay captured batches of this many steps
  hipStream_t cap_stream = nullptr;  // library-owned stream used only for capture
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0, graph_seg = 0, graph_key = 0;
  // two steps per pass: on, tiling its roles were built for, and whether
  // the two field sets have traded places (state n lives in set
  // (n & 1) ^ flip; a pair of launches writes step n+2 into the other set)
  bool tb = false;
  int tb_seg = 0;
  int pair_split = -1;   // percent of far tiles in a pair's second launch (-1: default)
  int flip = 0;
  // periodic finiteness check of the field set: every check_every steps
  // (0: never) run() launches finite_check_kernel; a run that launched one
  // synchronises and reports a non-finite value as FDTD_EUNSTABLE
  int check_every = 1024;
  int since_check = 0;
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_st, ev_cp;
  size_t used_st = 0, used_cp = 0;
  double ms_st = 0, ms_cp = 0;
  int64_t n_st = 0, n_cp = 0;
};

namespace fdtd {

// physical field set (0 or 1) holding the handle's current state
inline int cur_set(const fdtd_rom_sim* s) { return (s->steps & 1) ^ s->flip; }

template <typename T>
StepParams<T>& step_params(fdtd_rom_sim* s) {
  if constexpr (sizeof(T) == 4) return s->sp_f;
  else return s->sp_d;
}

// Shape-level validation and device workspace plan of one problem.
int plan_problem(const fdtd_problem* p, Layout& L);

// Advance the simulation by nsteps (graph replays or plain launches).
int run_steps_any(fdtd_rom_sim* s, int nsteps);
// The same with one plain launch per step only: no graph capture, no tile
// roles, no finiteness check, nothing allocated (bit-identical results).
int run_direct_any(fdtd_rom_sim* s, int nsteps);

// Rows per stencil wave: recompute the tile grid of the handle.
void set_tiling(fdtd_rom_sim* s, int seg);
// Rows per stencil wave a new handle starts with (grid size, element bytes).
int default_tiling(int nx, int ny, int ts);
// The same for the two-step launches.
int default_tiling2(int nx, int ny, int ts);
// Tile roles of the two-step launches for the handle's current tiling,
// uploaded synchronously on its stream (a no-op when already current).
template <typename T>
int prepare_tb(fdtd_rom_sim* s);

}  // namespace fdtd
