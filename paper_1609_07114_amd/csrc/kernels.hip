// gfx950 kernels of the embedded-ROM FDTD time step.
//
// One launch per leap-frog step n -> n+1 (step_kernel).  Its workgroups are
// of three kinds, all reading only the step-n buffers (set n & 1) and writing
// disjoint parts of the step-(n+1) buffers, so they run concurrently:
//   * coupling blocks (first, so they start early): eq. (23) for every
//     embedded model, written as one matrix G on z = [x~^n; h^{n+1/2}]
//     giving [x~^{n+1}; y^{n+1}] - a row-parallel GEMV per model, or, for
//     regions sharing one model (FP32), one MFMA GEMM over the copies.  h (the coarse Hz^{n+1/2} just outside the
//     ports) is recomputed from the step-n fields with the same arithmetic as
//     the stencil, so it equals the stencil's value bit for bit; y^{n+1} is
//     written into the interface edges;
//   * stencil tiles: coarse leap-frog update (eq. (5) then eq. (3)),
//     Hz^{n-1/2} -> Hz^{n+1/2}, E^n -> E^{n+1} on every edge that is neither
//     on a PEC wall nor on or inside a reduced region, plus additive sources;
//   * one probe block: records probe row n-1 (Hz^{n-1/2}, E^n), i.e. the
//     values the previous launch produced.
// A probe-flush launch records the last row of a batch and a one-thread tick
// launch advances the device step base.
//
// Stencil design (HBM-bound, one pass per step):
//   * a wave owns 64 adjacent columns and marches up a segment of SEG rows,
//     carrying Ex(i,j), Hz^{n+1/2}(i,j-1) and the material of row j-1 in
//     registers, with the loads of row j+1 issued before row j is computed;
//     horizontal neighbours (Ey(i+1,j), Hz^{n+1/2}(i-1,j), material of cell
//     i-1) come from adjacent lanes (DPP whole-wave shifts), lanes 0 and 63
//     fetch the one column outside the wave;
//   * each segment recomputes Hz^{n+1/2} of the row below it (one extra row
//     per SEG), so the step needs no second pass;
//   * per-edge coefficients are rebuilt from per-cell (a, b) =
//     (eps0*eps_r/dt, sigma/2): s = a1+a2, t = b1+b2, Ca = (s-t)/(s+t),
//     Cb/d = (2/d)/(s+t) - 32 algorithmic bytes per cell update instead of
//     the 40 a per-edge coefficient table would cost;
//   * cells inside a reduced region carry a < 0: their Hz stays zero, edges
//     inside keep their (zero) value and interface edges are not written;
//   * workgroups are remapped so each of the 8 XCDs (own L2) takes a
//     contiguous band of tiles, keeping the halo rows within one L2.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "device.hpp"

namespace fdtd {

__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int xcd = bid & 7;
  const int local = bid >> 3;
  const int per = nblk >> 3;
  const int rem = nblk & 7;
  return (xcd < rem) ? xcd * (per + 1) + local
                     : rem * (per + 1) + (xcd - rem) * per + local;
}

// eq. (5) divided by the cell area; shared by the stencil and the coupling
// blocks so both produce identical Hz^{n+1/2}
template <typename T>
__device__ __forceinline__ T hz_update(T h, T ex0, T ex1, T ey0, T ey1, T chdy, T chdx) {
#pragma clang fp contract(off)
  return h + (chdy * (ex1 - ex0) - chdx * (ey1 - ey0));
}

template <typename T>
__device__ __forceinline__ void edge_coef(T s, T t, T k2, T& ca, T& cb) {
#pragma clang fp contract(off)
  const T rcp = T(1) / (s + t);
  ca = (s - t) * rcp;
  cb = k2 * rcp;
}

// field pointer of set `par`, component c (selects, not dynamic indexing of
// the kernel-argument array)
template <typename T>
__device__ __forceinline__ T* fld(const StepParams<T>& p, int par, int c) {
  T* a = c == 0 ? p.f[0][0] : (c == 1 ? p.f[0][1] : p.f[0][2]);
  T* b = c == 0 ? p.f[1][0] : (c == 1 ? p.f[1][1] : p.f[1][2]);
  return par ? b : a;
}

template <typename T>
__device__ __forceinline__ T src_sum(const StepParams<T>& p, const T* sinc, int comp, int i,
                                     int j) {
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

template <typename T>
struct RowIn {
  T h, ex1, ey0, al, be;
};

// One lane's column of row j: Hz, Ex(j+1) (zero above the top row: `up` is
// wave-uniform), Ey, material.  Columns up to the 64-aligned pitch are
// inside the arrays (padding reads zero, material zero = inactive).
template <typename T>
__device__ __forceinline__ RowIn<T> load_row(const T* hz, const T* ex_up, const T* ey, const T* al,
                                             const T* be, uint32_t ob, bool up) {
  RowIn<T> r;
  r.h = ld(hz, ob);
  r.ex1 = T(0);
  if (up) r.ex1 = ld(ex_up, ob);
  r.ey0 = ld(ey, ob);
  r.al = ld(al, ob);
  r.be = ld(be, ob);
  return r;
}

// The same row with the material from the table: `id` is the cell's 16-bit
// material index, loaded earlier (see stencil_rows).
template <typename T>
__device__ __forceinline__ RowIn<T> load_row_tab(const T* hz, const T* ex_up, const T* ey,
                                                 const MatPair<T>* mt, uint32_t id, uint32_t ob, bool up) {
  RowIn<T> r;
  r.h = ld(hz, ob);
  r.ex1 = T(0);
  if (up) r.ex1 = ld(ex_up, ob);
  r.ey0 = ld(ey, ob);
  const MatPair<T> m = mt[id];
  r.al = m.a;
  r.be = m.b;
  return r;
}

// 16-bit material index of the cell at byte offset `ob` of a T-sized array
template <typename T>
__device__ __forceinline__ uint32_t mat_id(const uint16_t* mi, uint32_t ob) {
  return ld(mi, ob / (uint32_t)(sizeof(T) / sizeof(uint16_t)));
}

// eq. (5) with stretched derivatives inside absorbing layers: dex, dey the
// Yee differences, ik 1/kappa, ps the updated auxiliary fields.
template <typename T>
__device__ __forceinline__ T hz_update_pml(T h, T dex, T dey, T chdy, T chdx, T iky, T ikx, T psy, T psx) {
#pragma clang fp contract(off)
  return h + (chdy * (iky * dex + psy) - chdx * (ikx * dey + psx));
}

// eq. (3): E' = Ca E + (Cb/d) dH, not contracted, so that the plain update
// and the absorbing-layer update with identity profiles round alike
template <typename T>
__device__ __forceinline__ T e_update(T ca, T e, T cb, T dh) {
#pragma clang fp contract(off)
  return ca * e + cb * dh;
}

// psi' = b psi + a dF (recursive convolution of the stretched derivative)
template <typename T>
__device__ __forceinline__ T psi_next(T b, T psi, T a, T d) {
#pragma clang fp contract(off)
  return b * psi + a * d;
}

template <typename T, int SEG, bool PML, bool MIdx>
__device__ __forceinline__ void stencil_rows(const StepParams<T>& p, int t, int n) {
  const int par = n & 1;
  const T* hz = fld(p, par, 0);
  const T* ex = fld(p, par, 1);
  const T* ey = fld(p, par, 2);
  T* hzo = fld(p, par ^ 1, 0);
  T* exo = fld(p, par ^ 1, 1);
  T* eyo = fld(p, par ^ 1, 2);
  const int lane = threadIdx.x & (kWave - 1);
  // wave index as a scalar: every row condition below is wave-uniform
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = xcd_tile(t, p.nst_blocks);
  const int tx = tile % p.tiles_x;
  const int tyb = tile / p.tiles_x;
  const int iw = tx * kWave;
  const int i = iw + lane;
  const int j0 = (tyb * (kBlock / kWave) + wv) * SEG;
  const int j1 = min(j0 + SEG, p.ny);
  const int nx = p.nx;
  const int ny = p.ny;
  const int P = p.pitch;
  constexpr uint32_t ts = sizeof(T);
  const uint32_t row_b = (uint32_t)P * ts;
  // parameters in registers: p may live in global memory (batched launch),
  // where the field stores below would otherwise force reloads
  const T chdy = p.chdy, chdx = p.chdx, k2dy = p.k2dy, k2dx = p.k2dx;
  const T* al = p.al;
  const T* be = p.be;
  const T* ex_up = ex + P;  // Ex of the row above, same offset
  const bool in = i < nx;
  const bool has_left = (lane == 0) && (i >= 1);
  const int js = j0 > 0 ? j0 - 1 : 0;
  // wave-uniform: does any source touch columns [iw-1, iw+64) x rows [js, j1)?
  bool any_src = false;
  for (int s = 0; s < p.nsrc; ++s) {
    const Src<T>& S = p.src[s];
    any_src |= S.i0 < iw + kWave && S.i1 > iw - 1 && S.j0 < j1 && S.j1 > js;
  }
  T sinc[kMaxSrc];
#pragma unroll
  for (int s = 0; s < kMaxSrc; ++s) sinc[s] = T(0);
  if (any_src) {
#pragma unroll
    for (int s = 0; s < kMaxSrc; ++s)
      if (s < p.nsrc) sinc[s] = p.src[s].incr[n];
  }
  // absorbing layers: x profiles of this lane's column (and lane 0's left
  // neighbour), auxiliary fields of this step's parity
  T ikx_e = T(1), bx_e = T(1), ax_e = T(0), ikx_h = T(1), bx_h = T(1), ax_h = T(0);
  T ikx_hl = T(1), bx_hl = T(1), ax_hl = T(0);
  const T* psx_in = nullptr;
  const T* psy_in = nullptr;
  T* psx_out = nullptr;
  T* psy_out = nullptr;
  if constexpr (PML) {
    const int S = p.px_stride;
    ikx_e = p.px[i];
    bx_e = p.px[S + i];
    ax_e = p.px[2 * S + i];
    ikx_h = p.px[3 * S + i];
    bx_h = p.px[4 * S + i];
    ax_h = p.px[5 * S + i];
    if (has_left) {
      ikx_hl = p.px[3 * S + i - 1];
      bx_hl = p.px[4 * S + i - 1];
      ax_hl = p.px[5 * S + i - 1];
    }
    psx_in = par ? p.psi_h[1][0] : p.psi_h[0][0];
    psy_in = par ? p.psi_h[1][1] : p.psi_h[0][1];
    psx_out = par ? p.psi_h[0][0] : p.psi_h[1][0];
    psy_out = par ? p.psi_h[0][1] : p.psi_h[1][1];
  }

  uint32_t ob = ((uint32_t)js * (uint32_t)P + (uint32_t)i) * ts;
  // The wave's west and east neighbour columns (read by lanes 0 and 63) are
  // addressed at wave-uniform offsets and loaded by every lane, and the Ex
  // row above the top row is replaced by a read of the row itself, so all
  // loads of a row are unconditional: the loads in flight are the same on
  // every path and the waits the compiler places are exact.
  const bool west = iw > 0;
  const bool east = iw + kWave < nx;
  const uint32_t dW = (uint32_t)(west ? lane + 1 : lane) * ts;            // own column -> west column
  const uint32_t dE = (uint32_t)(east ? kWave - lane : 0) * ts;           // own column -> east column
  const uint32_t dEn = (uint32_t)(east ? 0 : lane) * ts;                  // ... or back to column iw
  const uint16_t* mi = p.mi;
  const MatPair<T>* mt = p.mt;
  struct RowSet {
    RowIn<T> c, w;
    T eyE;
  };
  // row at byte offset o; ids: the material indices of its own and west
  // cells.  Values that do not exist (Ex above the top row, the east column
  // of the last tile) are zeroed where they are used, not here: zeroing a
  // register whose load is still in flight would wait for it.
  auto fetch = [&](uint32_t o, bool up, uint32_t id, uint32_t idw) {
    RowSet r;
    const T* exr = up ? ex_up : ex;
    const uint32_t ow = o - dW;
    r.c.h = ld(hz, o);
    r.c.ex1 = ld(exr, o);
    r.c.ey0 = ld(ey, o);
    r.w.h = ld(hz, ow);
    r.w.ex1 = ld(exr, ow);
    r.w.ey0 = ld(ey, ow);
    r.eyE = ld(ey, o + dE - dEn);
    if constexpr (MIdx) {
      const MatPair<T> m = mt[id], mw = mt[idw];
      r.c.al = m.a;
      r.c.be = m.b;
      r.w.al = mw.a;
      r.w.be = mw.b;
    } else {
      r.c.al = ld(al, o);
      r.c.be = ld(be, o);
      r.w.al = ld(al, ow);
      r.w.be = ld(be, ow);
    }
    return r;
  };
  // row offset of row r (< j1)
  auto orow = [&](int r) { return ob + (uint32_t)(r - js) * row_b; };
  T ex_c = ld(ex, ob);
  T exl_c = ld(ex, ob - dW);  // used by lane 0 only when the west column exists
  T hn_prev = T(0), a_prev = T(0), b_prev = T(0);
  // software pipeline, two rows deep: rows j+1 and j+2 are in flight while
  // row j is computed.  With a material table the 16-bit indices run two
  // rows further ahead (loaded two iterations before their table gather),
  // so a gather never waits on a load issued after the rows it needs.
  uint32_t idA = 0, idB = 0, idAw = 0, idBw = 0;
  RowSet n1, n2;
  if constexpr (MIdx) {
    const uint32_t o0 = orow(js), o1 = orow(js + 1);
    const uint32_t oA = orow(min(js + 2, j1 - 1)), oB = orow(min(js + 3, j1 - 1));
    const uint32_t i0 = mat_id<T>(mi, o0), i0w = mat_id<T>(mi, o0 - dW);
    const uint32_t i1 = mat_id<T>(mi, o1), i1w = mat_id<T>(mi, o1 - dW);
    idA = mat_id<T>(mi, oA);
    idAw = mat_id<T>(mi, oA - dW);
    idB = mat_id<T>(mi, oB);
    idBw = mat_id<T>(mi, oB - dW);
    n1 = fetch(o0, js + 1 < ny, i0, i0w);
    n2 = fetch(o1, js + 2 < ny, i1, i1w);
  } else {
    n1 = fetch(orow(js), js + 1 < ny, 0, 0);
    n2 = fetch(orow(js + 1), js + 2 < ny, 0, 0);
  }
  // one row: compute row j from `cur` (own, west, east data of row j)
  auto compute = [&](int j, const RowSet& cs) {
    RowIn<T> cur = cs.c;
    RowIn<T> cul = cs.w;  // used by lane 0 only when the west column exists
    if (j + 1 >= ny) {
      cur.ex1 = T(0);
      cul.ex1 = T(0);
    }
    const T ey1_r = east ? cs.eyE : T(0);
    T ey1 = lane_next(cur.ey0);
    if (lane == kWave - 1) ey1 = ey1_r;
    // y profiles of this row (wave-uniform)
    T iky_h = T(1), by_h = T(1), ay_h = T(0), iky_e = T(1), by_e = T(1), ay_e = T(0);
    T psy = T(0), psx = T(0);
    if constexpr (PML) {
      const int S = p.py_stride;
      iky_e = p.py[j];
      by_e = p.py[S + j];
      ay_e = p.py[2 * S + j];
      iky_h = p.py[3 * S + j];
      by_h = p.py[4 * S + j];
      ay_h = p.py[5 * S + j];
    }
    // eq. (5): Hz^{n+1/2}
    T hn;
    if constexpr (PML) {
      const T dex = cur.ex1 - ex_c, dey = ey1 - cur.ey0;
      psy = psi_next(by_h, ld(psy_in, ob), ay_h, dex);
      psx = psi_next(bx_h, ld(psx_in, ob), ax_h, dey);
      hn = hz_update_pml(cur.h, dex, dey, chdy, chdx, iky_h, ikx_h, psy, psx);
    } else {
      hn = hz_update(cur.h, ex_c, cur.ex1, cur.ey0, ey1, chdy, chdx);
    }
    if (any_src) hn += src_sum(p, sinc, 0, i, j);
    if (!(cur.al > T(0))) hn = T(0);
    T hnl = lane_prev(hn);
    T all = lane_prev(cur.al);
    T bel = lane_prev(cur.be);
    if (lane == 0) {
      hnl = T(0);
      all = cul.al;
      bel = cul.be;
      if (has_left) {
        if constexpr (PML) {
          const T dex = cul.ex1 - exl_c, dey = cur.ey0 - cul.ey0;
          const T psyl = psi_next(by_h, ld(psy_in, ob - ts), ay_h, dex);
          const T psxl = psi_next(bx_hl, ld(psx_in, ob - ts), ax_hl, dey);
          hnl = hz_update_pml(cul.h, dex, dey, chdy, chdx, iky_h, ikx_hl, psyl, psxl);
        } else {
          hnl = hz_update(cul.h, exl_c, cul.ex1, cul.ey0, cur.ey0, chdy, chdx);
        }
        if (any_src) hnl += src_sum(p, sinc, 0, i - 1, j);
        if (!(all > T(0))) hnl = T(0);
        exl_c = cul.ex1;
      }
    }
    if (j >= j0) {
      // eq. (3), branch-free: both coefficients are formed on every lane and
      // the update is selected (a division by a non-positive sum on an edge
      // that is not updated is discarded)
      // Ex^{n+1}(i,j) between cells (i,j-1) and (i,j)
      const bool ax = j >= 1 && cur.al > T(0) && a_prev > T(0);
      T cax, cbx;
      edge_coef(cur.al + a_prev, cur.be + b_prev, k2dy, cax, cbx);
      // Ey^{n+1}(i,j) between cells (i-1,j) and (i,j)
      const bool ay = i >= 1 && cur.al > T(0) && all > T(0);
      T cay, cby;
      edge_coef(cur.al + all, cur.be + bel, k2dx, cay, cby);
      T exn, eyn, pex = T(0), pey = T(0);
      if constexpr (PML) {
        const T dhx = hn - hn_prev, dhy = hn - hnl;
        pex = psi_next(by_e, ld(p.psi_ex, ob), ay_e, dhx);
        pey = psi_next(bx_e, ld(p.psi_ey, ob), ax_e, dhy);
        exn = ax ? e_update(cax, ex_c, cbx, psi_next(iky_e, dhx, T(1), pex)) : ex_c;
        eyn = ay ? e_update(cay, cur.ey0, cby, -psi_next(ikx_e, dhy, T(1), pey)) : cur.ey0;
      } else {
        exn = ax ? e_update(cax, ex_c, cbx, hn - hn_prev) : ex_c;
        eyn = ay ? e_update(cay, cur.ey0, cby, -(hn - hnl)) : cur.ey0;
      }
      if (any_src) {
        exn += src_sum(p, sinc, 1, i, j);
        eyn += src_sum(p, sinc, 2, i, j);
      }
      if (in) {
        st(hzo, ob, hn);
        // interface edges (exactly one side inside a region) belong to the
        // coupling blocks of this launch
        if (!((cur.al < T(0)) != (a_prev < T(0)))) st(exo, ob, exn);
        if (!((cur.al < T(0)) != (all < T(0)))) st(eyo, ob, eyn);
        if constexpr (PML) {
          st(psy_out, ob, psy);
          st(psx_out, ob, psx);
          if (ax) st(p.psi_ex, ob, pex);
          if (ay) st(p.psi_ey, ob, pey);
        }
      }
    }
    hn_prev = hn;
    a_prev = cur.al;
    b_prev = cur.be;
    ex_c = cur.ex1;
  };
  int j = js;
  for (; j + 2 < j1; ++j, ob += row_b) {
    const RowSet cur = n1;
    n1 = n2;
    const uint32_t o3 = ob + 2 * row_b;
    if constexpr (MIdx) {
      const uint32_t oC = o3 + (j + 3 < j1 ? row_b : 0u) + (j + 4 < j1 ? row_b : 0u);
      const uint32_t idC = mat_id<T>(mi, oC), idCw = mat_id<T>(mi, oC - dW);
      n2 = fetch(o3, j + 3 < ny, idA, idAw);
      idA = idB;
      idAw = idBw;
      idB = idC;
      idBw = idCw;
    } else {
      n2 = fetch(o3, j + 3 < ny, 0, 0);
    }
    compute(j, cur);
  }
  for (; j < j1; ++j, ob += row_b) {
    const RowSet cur = n1;
    n1 = n2;
    compute(j, cur);
  }
}

// A stencil wave takes the absorbing-layer variant only when its columns
// [iw-1, iw+64) or rows [js, j1) reach into a layer.  Kernels built with
// Layers = false (problems without layers) contain the plain variant only,
// so its register budget is not raised by the layer code.
template <typename T, int SEG, bool Layers, bool MIdx>
__device__ __forceinline__ void stencil_tile(const StepParams<T>& p, int t, int n) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = xcd_tile(t, p.nst_blocks);
  const int iw = (tile % p.tiles_x) * kWave;
  const int j0 = ((tile / p.tiles_x) * (kBlock / kWave) + wv) * SEG;
  if (j0 >= p.ny) return;  // uniform over the wave: no rows left for it
  if constexpr (!Layers) {
    stencil_rows<T, SEG, false, MIdx>(p, t, n);
    return;
  }
  const int j1 = min(j0 + SEG, p.ny);
  const int js = j0 > 0 ? j0 - 1 : 0;
  const bool layer = p.pml && (iw - 1 < p.pml_xlo || iw + kWave > p.nx - p.pml_xhi ||
                               js < p.pml_ylo || j1 > p.ny - p.pml_yhi);
  if (layer)
    stencil_rows<T, SEG, true, MIdx>(p, t, n);
  else
    stencil_rows<T, SEG, false, MIdx>(p, t, n);
}

// ---------------------------------------------------------------------------
// Two steps per pass (time blocking) for grids without absorbing layers.
// A wave holds 64 lanes = columns iw-2 .. iw+61 (iw = kOwned2 * tile
// column) and makes one sweep up its rows doing two steps: stage 1 advances
// rows [rs, re] from step n to n+1 with exactly the arithmetic of
// stencil_rows; stage 2 trails one row behind and advances the stage-1 row
// below from n+1 to n+2 in registers.  Every horizontal neighbour comes from
// the adjacent lane, so the wave reads only its own 64 columns: stage-1
// values are exact on lanes 1..62 (lane 0 lacks its west Hz, lane 63 its
// east Ey), stage-2 values on lanes 2..61, which own their columns.  Stage-1
// rows [j0-2, j1] feed stage-2 rows [j0-1, j1), so only step n+2 goes to
// memory: 26 bytes per cell for two steps instead of 52.
//
// Near = false: a far tile, whose reads never reach a reduced region, its
//   ring or a source: two steps into f2, every owned sample stored.
// Near = true: a tile near a region or a source (first launch of the pair):
//   the same two steps with source terms, storing
//   * stage 1 (step n+1) into the step-(n+1) set where the second launch
//     reads it (StepParams::st1m: a box around each ring cell), except
//     interface edges (the step-n coupling writes them);
//   * stage 2 (step n+2) into f2, except the band around each region - the
//     Hz of ring cells (active cells with a side on a region cell) and E on
//     every edge of a ring cell - and the interface edges.  The band's step
//     n+2 depends on the step-(n+1) interface E of eq. (23), which only the
//     coupling blocks of this launch produce; the second launch's band
//     blocks compute it from the step-(n+1) set.
template <typename T>
struct RowIn2 {
  T h, ex1, ey0, al, be;
};

// stage-1 result of one row, kept for stage 2
template <typename T>
struct Stage1 {
  T h, ex, ey;              // Hz^{n+1/2}, Ex^{n+1}, Ey^{n+1}
  T cax, cbx, cay, cby;     // eq. (3) coefficients of the row's south Ex and west Ey
  bool act, ax, ay;         // active cell, updated edges
  bool ix, iy;              // south Ex / west Ey are interface edges (near tiles)
};

// The sets a two-step sweep reads (step n) and writes (step n+2; near
// tiles also step n+1)
template <typename T>
struct Sets2 {
  const T* hz;
  const T* ex;
  const T* ey;
  T* hzo;
  T* exo;
  T* eyo;
  T* hz1;
  T* ex1o;
  T* ey1o;
};

// The first launch's sets: step n is set n & 1, step n+1 the other (the
// third field set), step n+2 is f2.
template <typename T>
__device__ __forceinline__ Sets2<T> sets_first(const StepParams<T>& p, int n) {
  const int par = n & 1;
  return Sets2<T>{fld(p, par, 0), fld(p, par, 1), fld(p, par, 2), p.f2[0], p.f2[1], p.f2[2],
                  fld(p, par ^ 1, 0), fld(p, par ^ 1, 1), fld(p, par ^ 1, 2)};
}

// The second launch (its step index n is the pair's n+1): far tiles moved
// into it read the pair's step-n set, which the host passes as f2, and
// write the pair's output set, the set this launch's coupling writes.
template <typename T>
__device__ __forceinline__ Sets2<T> sets_second(const StepParams<T>& p, int n) {
  const int po = (n & 1) ^ 1;
  return Sets2<T>{p.f2[0], p.f2[1], p.f2[2], fld(p, po, 0), fld(p, po, 1), fld(p, po, 2), nullptr, nullptr, nullptr};
}

template <typename T, bool MIdx, bool Near>
__device__ __forceinline__ void stencil2_rows(const StepParams<T>& p, const Sets2<T>& S, int tile, int n, int j0,
                                              int j1) {
  const T* hz = S.hz;
  const T* ex = S.ex;
  const T* ey = S.ey;
  T* hzo = S.hzo;
  T* exo = S.exo;
  T* eyo = S.eyo;
  // near tiles: the step-(n+1) set receives stage 1
  T* hz1 = S.hz1;
  T* ex1o = S.ex1o;
  T* ey1o = S.ey1o;
  const int lane = threadIdx.x & (kWave - 1);
  const int iw = (tile % p.tiles_x2) * kOwned2;
  const int c = iw - 2 + lane;
  const int nx = p.nx, ny = p.ny, P = p.pitch;
  // stage-1 rows [rs, re]
  const int rs = max(j0 - 2, 0);
  const int re = min(j1, ny - 1);
  const int r2lo = max(j0 - 1, 0);  // first stage-2 row (its Hz only, unless j0 = 0)
  constexpr uint32_t ts = sizeof(T);
  const uint32_t row_b = (uint32_t)P * ts;
  const T chdy = p.chdy, chdx = p.chdx, k2dy = p.k2dy, k2dx = p.k2dx;
  const T* al = p.al;
  const T* be = p.be;
  const T* ex_up = ex + P;
  const bool in = c >= 0 && c < nx;
  const bool own = in && lane >= 2 && lane <= kWave - 3;
  // sources touching columns [iw-2, iw+62) x rows [rs, re]; far tiles have
  // none in reach (sources make a tile near), so their code holds no source
  // terms and keeps the register count of the two-step sweep down
  bool any_src = false;
  if constexpr (Near) {
    for (int s = 0; s < p.nsrc; ++s) {
      const Src<T>& S = p.src[s];
      any_src |= S.i0 < iw + kWave - 2 && S.i1 > iw - 2 && S.j0 <= re && S.j1 > rs;
    }
  }
  T sinc[kMaxSrc], sinc2[kMaxSrc];  // increments of steps n and n+1
#pragma unroll
  for (int s = 0; s < kMaxSrc; ++s) sinc[s] = sinc2[s] = T(0);
  if (any_src) {
#pragma unroll
    for (int s = 0; s < kMaxSrc; ++s)
      if (s < p.nsrc) {
        sinc[s] = p.src[s].incr[n];
        sinc2[s] = p.src[s].incr[n + 1];
      }
  }
  // the lane's column, clamped into the row: lanes outside the grid read a
  // valid address and their values are never used
  const int cl = min(max(c, 0), P - 1);
  uint32_t ob = ((uint32_t)rs * (uint32_t)P + (uint32_t)cl) * ts;
  const uint16_t* mi = p.mi;
  const MatPair<T>* mt = p.mt;
  auto fetch = [&](uint32_t o, bool up, uint32_t id) {
    RowIn2<T> r;
    r.h = ld(hz, o);
    r.ex1 = ld(up ? ex_up : ex, o);
    r.ey0 = ld(ey, o);
    if constexpr (MIdx) {
      const MatPair<T> m = mt[id];
      r.al = m.a;
      r.be = m.b;
    } else {
      r.al = ld(al, o);
      r.be = ld(be, o);
    }
    return r;
  };
  auto orow = [&](int r) { return ob + (uint32_t)(r - rs) * row_b; };
  T ex_c = ld(ex, ob);
  T hn_prev = T(0), a_prev = T(0), b_prev = T(0);
  T a_prev2 = T(0);     // near tiles: material a of the row below the stage-2 row
  bool ring_prev = false;  // near tiles: the row below the stage-2 row is a ring cell
  Stage1<T> prv1{};
  T h2_prev = T(0);
  // stage 2 for row r2 from its stage-1 values `a` and Ex^{n+1} of the row
  // above (exN), stored at byte offset o2; near tiles also take the
  // material a of the cells at and around (c, r2) to find the band
  auto stage2 = [&](int r2, const Stage1<T>& a, T exN, uint32_t o2, T a_c, T a_up) {
    T eye = lane_next(a.ey);
    if (c + 1 >= nx) eye = T(0);
    T h2 = hz_update(a.h, a.ex, exN, a.ey, eye, chdy, chdx);
    if (any_src) h2 += src_sum(p, sinc2, 0, c, r2);
    if (!a.act) h2 = T(0);
    const T h2w = lane_prev(h2);
    bool ring = false, ring_w = false;
    if constexpr (Near) {
      ring = a_c > T(0) && (a_prev2 < T(0) || a_up < T(0) || lane_prev(a_c) < T(0) || lane_next(a_c) < T(0));
      ring_w = dpp_prev(ring ? 1 : 0) != 0;
    }
    if (r2 >= j0 && own) {
      T ex2 = a.ax ? e_update(a.cax, a.ex, a.cbx, h2 - h2_prev) : a.ex;
      T ey2 = a.ay ? e_update(a.cay, a.ey, a.cby, -(h2 - h2w)) : a.ey;
      if constexpr (Near) {
        if (any_src) {
          ex2 += src_sum(p, sinc2, 1, c, r2);
          ey2 += src_sum(p, sinc2, 2, c, r2);
        }
        if (!ring) st(hzo, o2, h2);
        if (!(ring || ring_prev || a.ix)) st(exo, o2, ex2);
        if (!(ring || ring_w || a.iy)) st(eyo, o2, ey2);
      } else {
        // far tiles have no interface edges in reach: every edge is stored
        st(hzo, o2, h2);
        st(exo, o2, ex2);
        st(eyo, o2, ey2);
      }
    }
    h2_prev = h2;
    if constexpr (Near) {
      ring_prev = ring;
      a_prev2 = a_c;
    }
  };
  // stage 1 for row r from its loaded data
  auto compute = [&](int r, const RowIn2<T>& cs) {
    RowIn2<T> cur = cs;
    if (r + 1 >= ny) cur.ex1 = T(0);
    T ey1 = lane_next(cur.ey0);
    if (c + 1 >= nx) ey1 = T(0);
    const bool act = in && cur.al > T(0);
    T hn = hz_update(cur.h, ex_c, cur.ex1, cur.ey0, ey1, chdy, chdx);
    if (any_src) hn += src_sum(p, sinc, 0, c, r);
    if (!act) hn = T(0);
    const T hnl = lane_prev(hn);
    const T all = lane_prev(cur.al);
    const T bel = lane_prev(cur.be);
    Stage1<T> o;
    o.act = act;
    o.ax = r >= 1 && act && a_prev > T(0);
    edge_coef(cur.al + a_prev, cur.be + b_prev, k2dy, o.cax, o.cbx);
    o.ay = c >= 1 && act && all > T(0);
    edge_coef(cur.al + all, cur.be + bel, k2dx, o.cay, o.cby);
    T exn = o.ax ? e_update(o.cax, ex_c, o.cbx, hn - hn_prev) : ex_c;
    T eyn = o.ay ? e_update(o.cay, cur.ey0, o.cby, -(hn - hnl)) : cur.ey0;
    if (any_src) {
      exn += src_sum(p, sinc, 1, c, r);
      eyn += src_sum(p, sinc, 2, c, r);
    }
    o.h = hn;
    o.ex = exn;
    o.ey = eyn;
    o.ix = o.iy = false;
    if constexpr (Near) {
      // interface edges (exactly one side inside a region) belong to the
      // coupling blocks
      o.ix = (cur.al < T(0)) != (a_prev < T(0));
      o.iy = (cur.al < T(0)) != (all < T(0));
      // only where the second launch reads the step-(n+1) set
      if (own && r >= j0 && r < j1 && p.st1m[ob / ts] != 0) {
        st(hz1, ob, hn);
        if (!o.ix) st(ex1o, ob, exn);
        if (!o.iy) st(ey1o, ob, eyn);
      }
    }
    if (r - 1 >= r2lo) stage2(r - 1, prv1, exn, ob - row_b, a_prev, cur.al);
    else if constexpr (Near) a_prev2 = a_prev;  // rows below the first stage-2 row
    prv1 = o;
    hn_prev = hn;
    a_prev = cur.al;
    b_prev = cur.be;
    ex_c = cur.ex1;
  };
  // software pipeline as in stencil_rows: rows r+1 and r+2 in flight while
  // row r is computed; material indices two rows further ahead
  const int rend = re + 1;
  uint32_t idA = 0, idB = 0;
  RowIn2<T> n1, n2;
  if constexpr (MIdx) {
    const uint32_t o0 = orow(rs), o1 = orow(min(rs + 1, re));
    const uint32_t i0 = mat_id<T>(mi, o0), i1 = mat_id<T>(mi, o1);
    idA = mat_id<T>(mi, orow(min(rs + 2, re)));
    idB = mat_id<T>(mi, orow(min(rs + 3, re)));
    n1 = fetch(o0, rs + 1 < ny, i0);
    n2 = fetch(o1, rs + 2 < ny, i1);
  } else {
    n1 = fetch(orow(rs), rs + 1 < ny, 0);
    n2 = fetch(orow(min(rs + 1, re)), rs + 2 < ny, 0);
  }
  int r = rs;
  for (; r + 2 < rend; ++r, ob += row_b) {
    const RowIn2<T> cur = n1;
    n1 = n2;
    const uint32_t o3 = ob + 2 * row_b;
    if constexpr (MIdx) {
      const uint32_t oC = o3 + (r + 3 < rend ? row_b : 0u) + (r + 4 < rend ? row_b : 0u);
      const uint32_t idC = mat_id<T>(mi, oC);
      n2 = fetch(o3, r + 3 < ny, idA);
      idA = idB;
      idB = idC;
    } else {
      n2 = fetch(o3, r + 3 < ny, 0);
    }
    compute(r, cur);
  }
  for (; r < rend; ++r, ob += row_b) {
    const RowIn2<T> cur = n1;
    n1 = n2;
    compute(r, cur);
  }
  // the top row of the grid: its stage 2 has the north wall above it
  if (j1 == ny) stage2(ny - 1, prv1, T(0), ob - row_b, a_prev, T(0));
}

// Second launch of a pair, part `part` of region k's band, step n (the
// pair's second step): the band around the region - Hz of every ring cell
// (the coarse cell outside each port) and E on its edges other than
// interface edges - advanced from the step-n set (stage-1 values of the
// near tiles, interface E of the first launch's coupling) into the
// step-(n+1) set with the stencil's arithmetic.  Hz^{n+1/2} of a ring cell
// and of its neighbours is formed from the step-n set as the stencil forms
// it (ring_h), so every value equals the one a single-step launch would
// produce; an edge shared by two ring cells is formed by both, equal bit for
// bit.  A region's 5 np samples (Hz and four edges per port) are dealt to
// kBandSplit workgroups.
template <typename T>
__device__ __forceinline__ void band_block(const StepParams<T>& p, int k, int part, int n) {
  const int par = n & 1;
  const T* hz = fld(p, par, 0);
  const T* ex = fld(p, par, 1);
  const T* ey = fld(p, par, 2);
  T* hzo = fld(p, par ^ 1, 0);
  T* exo = fld(p, par ^ 1, 1);
  T* eyo = fld(p, par ^ 1, 2);
  const RomDev r = p.roms[k];
  const int* gi = p.idx + r.i_off;
  const int P = p.pitch;
  auto mat = [&](int oc, T& a, T& b) {
    if (p.midx) {
      const MatPair<T> m = p.mt[p.mi[oc]];
      a = m.a;
      b = m.b;
    } else {
      a = p.al[oc];
      b = p.be[oc];
    }
  };
  auto srcs = [&](int comp, int ii, int jj) {
    T acc = T(0);
    for (int s = 0; s < p.nsrc; ++s) {
      const Src<T>& S = p.src[s];
      if (S.comp == comp && ii >= S.i0 && ii < S.i1 && jj >= S.j0 && jj < S.j1) acc += S.incr[n];
    }
    return acc;
  };
  const int items = 5 * r.np;
  const int per = (items + kBandSplit - 1) / kBandSplit;
  const int u1 = min(items, (part + 1) * per);
  for (int u = part * per + threadIdx.x; u < u1; u += kBlock) {
    const int port = u / 5, what = u - 5 * port;
    const int o = gi[port];
    const int j = o / P, i = o - j * P;
    if (what == 0) {
      T a, b;
      mat(o, a, b);
      hzo[o] = a > T(0) ? ring_h(p, hz, ex, ey, o, n) : T(0);
      continue;
    }
    // edge between cells lo (south / west) and hi (north / east)
    const bool isx = what <= 2;
    const int hi = what == 1 ? o : what == 2 ? o + P : what == 3 ? o : o + 1;
    const int lo = isx ? hi - P : hi - 1;
    const int ei = isx ? i : (what == 3 ? i : i + 1);
    const int ej = isx ? (what == 1 ? j : j + 1) : j;
    if (isx ? (ej < 1 || ej > p.ny - 1) : (ei < 1 || ei > p.nx - 1)) continue;  // a wall
    T a_hi, b_hi, a_lo, b_lo;
    mat(hi, a_hi, b_hi);
    mat(lo, a_lo, b_lo);
    if ((a_hi < T(0)) != (a_lo < T(0))) continue;  // an interface edge: the coupling's
    T v = isx ? ex[hi] : ey[hi];
    if (a_hi > T(0) && a_lo > T(0)) {
      T ca, cb;
      edge_coef(a_hi + a_lo, b_hi + b_lo, isx ? p.k2dy : p.k2dx, ca, cb);
      const T d = ring_h(p, hz, ex, ey, hi, n) - ring_h(p, hz, ex, ey, lo, n);
      v = isx ? e_update(ca, v, cb, d) : e_update(ca, v, cb, -d);
    }
    if (p.nsrc > 0) v += srcs(isx ? 1 : 2, ei, ej);
    (isx ? exo : eyo)[hi] = v;
  }
}

// Far tiles of a pair: [0, far_split) go in the first launch, the rest in
// the second (both only read step n and write step n+2, so either launch
// may take them; the share in the second launch runs beside its coupling
// blocks, whose chain of dependent loads would otherwise be alone there).
// Workgroup t takes far slot t of its launch (XCD-remapped), wave w its rows
// [j0, j0+SEG); a near tile in that slot returns (its pieces run
// separately).
template <typename T, int SEG, bool MIdx, bool Second>
__device__ __forceinline__ void stencil2_tile(const StepParams<T>& p, int t, int n) {
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lo = Second ? p.far_split : 0, cnt = Second ? p.nst2_blocks - p.far_split : p.far_split;
  const int tile = lo + xcd_tile(t, cnt);
  if (p.role2[tile]) return;
  const int j0 = ((tile / p.tiles_x2) * (kBlock / kWave) + wv) * SEG;
  if (j0 >= p.ny) return;  // uniform over the wave
  stencil2_rows<T, MIdx, false>(p, Second ? sets_second(p, n) : sets_first(p, n), tile, Second ? n - 1 : n, j0,
                                min(j0 + SEG, p.ny));
}

// First launch, near tiles: each is split over pieces of near_rows-row waves.
// Their sweep does more per row than a far tile's (stage-1 stores, source
// terms, the band test); where the whole grid is resident at once the
// longest wave sets the launch's length, so near waves are kept short there
// (near_rows = 2), while larger grids keep whole tiles (less halo reread).
template <typename T, int SEG, bool MIdx>
__device__ __forceinline__ void stencil2_near(const StepParams<T>& p, int u, int n) {
  const int rows = min(p.near_rows, SEG);
  const int pieces = SEG / rows;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = p.near_list[u / pieces];
  const int jb0 = (tile / p.tiles_x2) * (kBlock / kWave) * SEG;
  const int jb1 = min(jb0 + (kBlock / kWave) * SEG, p.ny);
  const int j0 = jb0 + ((u % pieces) * (kBlock / kWave) + wv) * rows;
  if (j0 >= jb1) return;  // uniform over the wave
  stencil2_rows<T, MIdx, true>(p, sets_first(p, n), tile, n, j0, min(j0 + rows, jb1));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Coarse Hz^{n+1/2} of an active cell from the step-n fields (the value the
// stencil computes for it).
template <typename T>
__device__ __forceinline__ T ring_h(const StepParams<T>& p, const T* hz, const T* ex, const T* ey, int off, int n) {
  const int P = p.pitch;
  const int j = off / P;
  const int i = off - j * P;
  const T ex1 = (j + 1 < p.ny) ? ex[off + P] : T(0);
  const T ey1 = (i + 1 < p.nx) ? ey[off + 1] : T(0);
  T h = hz_update(hz[off], ex[off], ex1, ey[off], ey1, p.chdy, p.chdx);
  T acc = T(0);  // same summation order as the stencil's source term
  for (int s = 0; s < p.nsrc; ++s) {
    const Src<T>& S = p.src[s];
    if (S.comp == 0 && i >= S.i0 && i < S.i1 && j >= S.j0 && j < S.j1) acc += S.incr[n];
  }
  return p.nsrc > 0 ? h + acc : h;
}

// Rows [row0, row0 + kRowsPerBlock) of one model's eq. (23) update matrix.
template <typename T>
__device__ __forceinline__ void coupling_rows(const StepParams<T>& p, const RowBlock& rb, int n, T* z) {
  const int par = n & 1;
  const int tid = threadIdx.x;
  const RomDev r = p.roms[rb.a];
  const T* xin = p.xs + r.x_off + par * r.xstride;
  T* xout = p.xs + r.x_off + (par ^ 1) * r.xstride;
  const int* gi = p.idx + r.i_off;
  const int* si = gi + r.np;
  const T* hz = fld(p, par, 0);
  const T* ex = fld(p, par, 1);
  const T* ey = fld(p, par, 2);
  const int lane = tid & (kWave - 1);
  const int row0 = rb.b + (tid / kWave) * kRowsPerWave;
  const T* G = p.mats + r.g_off + (size_t)row0 * r.ldg;
  T acc[kRowsPerWave];
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) acc[k] = T(0);
  // z = [x~^n; h^{n+1/2}; 0] in LDS: reduced-state loads four rounds at a
  // time, then the ring Hz, then the padding
  auto stage = [&]() {
    for (int c0 = 0; c0 < r.q; c0 += 4 * kBlock) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * kBlock + tid;
        v[u] = c < r.q ? xin[c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u * kBlock + tid;
        if (c < r.q) z[c] = v[u];
      }
    }
    for (int c = r.q + tid; c < r.q + r.np; c += kBlock) z[c] = ring_h(p, hz, ex, ey, gi[c - r.q], n);
    for (int c = r.q + r.np + tid; c < r.ldg; c += kBlock) z[c] = T(0);
    lds_barrier();
  };
  lane_row_dots<T, kRowsPerWave>(G, r.ldg, z, lane, acc, stage);
#pragma unroll
  for (int k = 0; k < kRowsPerWave; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
    T* exo = fld(p, par ^ 1, 1);
    T* eyo = fld(p, par ^ 1, 2);
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
      const int row = row0 + k;
      if (row < r.q) {
        xout[row] = acc[k];
      } else if (row < r.q + r.np) {
        const int pp = row - r.q;
        if (pp < r.n_ex)
          exo[si[pp]] = acc[k];
        else
          eyo[si[pp]] = acc[k];
      }
    }
  }
}

// Shared model, many copies: Out (M x copies) = G (M x M) * Z (M x copies)
// with Z's column c = [x~_c^n; h_c^{n+1/2}] of region copies[b + c], as FP32
// MFMA 16x16x4 tiles.  Z is staged in LDS ([k][copy], 16 copies per row);
// a workgroup produces 64 output rows, each wave one 16-row tile, walking K
// in steps of 4 (short blocks: their chains of dependent loads run while
// the stencil tiles keep HBM busy).  Operand layout of v_mfma_f32_16x16x4f32
// (wave64): lane l holds A(l % 16, l / 16) and B(l / 16, l % 16); the
// result register i of lane l is D(4 * (l / 16) + i, l % 16).
__device__ __forceinline__ void coupling_gemm(const StepParams<float>& p, const RowBlock& gb, int n, float* zs) {
  const int par = n & 1;
  const int tid = threadIdx.x;
  const int ncp = gb.c;
  const int* list = p.copies + gb.b;
  const int M = p.roms[list[0]].ldg;  // padded q + np (multiple of 64), same for every copy
  const int64_t gt_off = p.roms[list[0]].gt_off;
  const float* hz = fld(p, par, 0);
  const float* ex = fld(p, par, 1);
  const float* ey = fld(p, par, 2);
  // Every thread owns one copy column c = tid % 16 for the whole block: its
  // descriptor is loaded once, and c is also the result column this thread's
  // lane holds after the MFMA loop (lane % 16), so the scatter reuses it.
  const int c = tid & (kGemmCopies - 1);
  const bool has = c < ncp;
  RomDev rc{};
  if (has) rc = p.roms[list[c]];
  const float* xin = p.xs + rc.x_off + par * rc.xstride;
  const int* gi = p.idx + rc.i_off;
#pragma unroll 4
  for (int k = tid / kGemmCopies; k < M; k += kBlock / kGemmCopies) {
    float v = 0.f;
    if (has) {
      if (k < rc.q)
        v = xin[k];
      else if (k < rc.q + rc.np)
        v = ring_h(p, hz, ex, ey, gi[k - rc.q], n);
    }
    zs[k * kGemmCopies + c] = v;
  }
  __syncthreads();
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int lr = lane & 15;  // A row / B column / D column within the tile (== c)
  const int lk = lane >> 4;  // A column / B row / D row group
  const float* GT = p.mats + gt_off;
  float* exo = fld(p, par ^ 1, 1);
  float* eyo = fld(p, par ^ 1, 2);
  float* xout = p.xs + rc.x_off + (par ^ 1) * rc.xstride;
  const int* si = gi + rc.np;
  const int rt = gb.a + wv;  // this wave's 16-row output tile
  if (rt < M / 16) {
    const int row0 = rt * 16;
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* a_ptr = GT + (size_t)lk * M + row0 + lr;
    const float* b_ptr = zs + lk * kGemmCopies + lr;
#pragma unroll 16
    for (int k0 = 0; k0 < M; k0 += 4) {
      const float a = a_ptr[(size_t)k0 * M];
      const float b = b_ptr[k0 * kGemmCopies];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    if (has) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = row0 + 4 * lk + i;
        if (row < rc.q) {
          xout[row] = acc[i];
        } else if (row < rc.q + rc.np) {
          const int pp = row - rc.q;
          if (pp < rc.n_ex)
            exo[si[pp]] = acc[i];
          else
            eyo[si[pp]] = acc[i];
        }
      }
    }
  }
}

// Probe row m (m >= 0) from the set holding the state after m+1 steps.
template <typename T>
__device__ __forceinline__ void record_probes(const StepParams<T>& p, int m) {
  if (m < 0) return;
  const int par = (m + 1) & 1;
  for (int t = threadIdx.x; t < p.nprobes; t += kBlock) {
    const int c = p.probe_comp[t];
    const int o = p.probe_off[t];
    p.probe_buf[(size_t)m * p.nprobes + t] = fld(p, par, c)[o];
  }
}

template <typename T, int SEG, bool Layers, bool MIdx>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !Layers ? 8 : 1, 8)))
step_kernel(const StepParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = p.ctrl[0] + p.step_off;
  const int b = blockIdx.x;
  if (b < p.ncoup_blocks) {
    if (b < p.nrowblocks) {
      const RowBlock rb = p.blocks[b];
      if constexpr (sizeof(T) == 4) {
        if (rb.kind == 1) {
          coupling_gemm(p, rb, n, reinterpret_cast<float*>(smem));
          return;
        }
      }
      coupling_rows(p, rb, n, reinterpret_cast<T*>(smem));
    }
    return;
  }
  const int t = b - p.ncoup_blocks;
  if (t < p.nst_blocks) {
    stencil_tile<T, SEG, Layers, MIdx>(p, t, n);
    return;
  }
  record_probes(p, n - 1);
}

// Value of probe t after step n+1 from the step-n set, formed exactly as the
// stencil forms it (its cell and neighbours are ordinary coarse cells: only
// probes of far tiles come here).
template <typename T>
__device__ __forceinline__ T probe_next(const StepParams<T>& p, int t, int n) {
  const int par = n & 1;
  const T* hz = fld(p, par, 0);
  const T* ex = fld(p, par, 1);
  const T* ey = fld(p, par, 2);
  const int P = p.pitch;
  const int o = p.probe_off[t];
  const int j = o / P;
  const int i = o - j * P;
  auto mat = [&](int oc, T& a, T& b) {
    if (p.midx) {
      const MatPair<T> m = p.mt[p.mi[oc]];
      a = m.a;
      b = m.b;
    } else {
      a = p.al[oc];
      b = p.be[oc];
    }
  };
  auto srcs = [&](int comp, int ii, int jj) {
    T acc = T(0);
    for (int s = 0; s < p.nsrc; ++s) {
      const Src<T>& S = p.src[s];
      if (S.comp == comp && ii >= S.i0 && ii < S.i1 && jj >= S.j0 && jj < S.j1) acc += S.incr[n];
    }
    return acc;
  };
  auto hnext = [&](int ii, int jj) {
    const int oc = jj * P + ii;
    const T ex1 = jj + 1 < p.ny ? ex[oc + P] : T(0);
    const T ey1 = ii + 1 < p.nx ? ey[oc + 1] : T(0);
    T h = hz_update(hz[oc], ex[oc], ex1, ey[oc], ey1, p.chdy, p.chdx);
    if (p.nsrc > 0) h += srcs(0, ii, jj);
    T a, b;
    mat(oc, a, b);
    return a > T(0) ? h : T(0);
  };
  const int comp = p.probe_comp[t];
  if (comp == 0) return hnext(i, j);
  T a, b, a2 = T(0), b2 = T(0);
  mat(o, a, b);
  T v = comp == 1 ? ex[o] : ey[o];
  const bool edge = comp == 1 ? j >= 1 : i >= 1;
  if (edge) mat(comp == 1 ? o - P : o - 1, a2, b2);
  if (edge && a > T(0) && a2 > T(0)) {
    T ca, cb;
    edge_coef(a + a2, b + b2, comp == 1 ? p.k2dy : p.k2dx, ca, cb);
    const T h = hnext(i, j);
    v = comp == 1 ? e_update(ca, v, cb, h - hnext(i, j - 1)) : e_update(ca, v, cb, -(h - hnext(i - 1, j)));
  }
  if (p.nsrc > 0) v += srcs(comp, i, j);
  return v;
}

// Probe block of a pair's first launch: row n-1 from the step-n set and
// row n formed from step n (every probe: none sits on an interface edge).
template <typename T>
__device__ __forceinline__ void pair_probes(const StepParams<T>& p, int n) {
  record_probes(p, n - 1);
  for (int k = threadIdx.x; k < p.nprobes; k += kBlock)
    p.probe_buf[(size_t)n * p.nprobes + k] = probe_next(p, k, n);
}

// The pair of launches that advances steps n and n+1 (time blocking):
//   first (Second = false): coupling blocks of step n (interface E^{n+1} into
//     the step-(n+1) set), every tile (far: two steps into f2; near: two
//     steps into f2 but for the band around each region, and step n+1 of
//     its cells into the step-(n+1) set), probe block (row n-1 from the
//     step-n set; row n formed from the step-n set);
//   second: coupling blocks of step n+1 (reading the step-(n+1) set, writing
//     f2's interface edges) and one band block per region (the band's step
//     n+1 -> n+2 into f2, here f[(n+1)&1 ^ 1]).
// FP32: eight waves per SIMD (the scalar registers the near tiles' source
// terms take would otherwise hold it to seven; the compiler keeps them in
// vector lanes, no scratch)
template <typename T, int SEG, bool MIdx, bool Second>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1, 8)))
step2_kernel(const StepParams<T> p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = p.ctrl[0] + p.step_off;
  const int b = blockIdx.x;
  if (b < p.ncoup_blocks) {
    if (b < p.nrowblocks) {
      const RowBlock rb = p.blocks[b];
      if constexpr (sizeof(T) == 4) {
        if (rb.kind == 1) {
          coupling_gemm(p, rb, n, reinterpret_cast<float*>(smem));
          return;
        }
      }
      coupling_rows(p, rb, n, reinterpret_cast<T*>(smem));
    }
    return;
  }
  const int t = b - p.ncoup_blocks;
  if constexpr (Second) {
    // band blocks padded to a multiple of 8 workgroups (XCD remap of the
    // far tiles that follow)
    const int nb = p.n_band * kBandSplit, nb8 = (nb + 7) & ~7;
    if (t < nb8) {
      // remapped like the near pieces: a region's parts on one XCD
      const int u = xcd_tile(t, nb8);
      if (u < nb) band_block(p, u / kBandSplit, u % kBandSplit, n);
    } else {
      stencil2_tile<T, SEG, MIdx, true>(p, t - nb8, n);
    }
  } else {
    // near pieces padded to a multiple of 8 workgroups, so that the far
    // tiles' XCD remap still sees workgroup t on XCD t % 8; the pieces are
    // remapped the same way (each XCD a contiguous run of the near list, so
    // a region's near tiles, which share halo rows and lines, share an L2)
    const int nn = p.n_near * (SEG / min(p.near_rows, SEG)), nn8 = (nn + 7) & ~7;
    if (t < nn8) {
      const int u = xcd_tile(t, nn8);
      if (u < nn) stencil2_near<T, SEG, MIdx>(p, u, n);
    } else if (t < nn8 + p.far_split) {
      stencil2_tile<T, SEG, MIdx, false>(p, t - nn8, n);
    } else {
      pair_probes(p, n);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) probe_kernel(const StepParams<T> p) {
  record_probes(p, p.ctrl[0] + p.step_off - 1);
}

__global__ void tick_kernel(int* ctrl, int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl[0] += k;
}

// Any non-finite value among n elements of a field set (n a multiple of the
// 16-byte vector width, the base 16-byte aligned): grid-stride 16-byte loads;
// a thread that finds one stores 1 into *flag (every writer stores the same
// value, so no atomics are needed; the host clears the flag).
template <typename T>
__global__ void __launch_bounds__(kBlock) finite_check_kernel(const T* __restrict__ f, size_t n, int* flag) {
  using V = std::conditional_t<sizeof(T) == 4, float4, double2>;
  constexpr int W = 16 / sizeof(T);
  const V* v = reinterpret_cast<const V*>(f);
  const size_t nv = n / W;
  bool bad = false;
  for (size_t k = (size_t)blockIdx.x * kBlock + threadIdx.x; k < nv; k += (size_t)gridDim.x * kBlock) {
    const V x = v[k];
    if constexpr (sizeof(T) == 4)
      bad |= !(__builtin_isfinite(x.x) && __builtin_isfinite(x.y) && __builtin_isfinite(x.z) &&
               __builtin_isfinite(x.w));
    else
      bad |= !(__builtin_isfinite(x.x) && __builtin_isfinite(x.y));
  }
  if (bad) flag[0] = 1;
}

// Batched step: B independent problems advance one step in one launch.
// Workgroup b takes table[b] = (instance, role, index) and runs the same
// device code as step_kernel on that instance's parameter block, which
// stays in global memory (read through the scalar cache).  Each instance
// keeps its own tile height.
template <typename T, bool Layers, bool MIdx>
__global__ void __launch_bounds__(kBlock)
batch_step_kernel(const StepParams<T>* __restrict__ descs, const BatchRef* __restrict__ table,
                  const int* __restrict__ ctrl, int step_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BatchRef r = table[blockIdx.x];
  if (r.kind == 3) return;
  const StepParams<T>& p = descs[r.inst];
  const int n = ctrl[0] + step_off;
  if (r.kind == 0) {
    const RowBlock rb = p.blocks[r.idx];
    if constexpr (sizeof(T) == 4) {
      if (rb.kind == 1) {
        coupling_gemm(p, rb, n, reinterpret_cast<float*>(smem));
        return;
      }
    }
    coupling_rows(p, rb, n, reinterpret_cast<T*>(smem));
    return;
  }
  if (r.kind == 1) {
    switch (p.seg) {
      case 4: stencil_tile<T, 4, Layers, MIdx>(p, r.idx, n); break;
      case 8: stencil_tile<T, 8, Layers, MIdx>(p, r.idx, n); break;
      case 32: stencil_tile<T, 32, Layers, MIdx>(p, r.idx, n); break;
      default: stencil_tile<T, 16, Layers, MIdx>(p, r.idx, n); break;
    }
    return;
  }
  record_probes(p, n - 1);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
batch_probe_kernel(const StepParams<T>* __restrict__ descs, const int* __restrict__ ctrl, int step_off) {
  record_probes(descs[blockIdx.x], ctrl[0] + step_off - 1);
}

// Batched pair launch: as batch_step_kernel, with the roles of the pair
// launches (kind 1: far two-step tiles of the first launch, band blocks of
// the second; kind 4: near-tile pieces of the first launch; kind 5: far
// tiles of the second launch; kind 2: the first launch's probe block).
template <typename T, bool MIdx, bool Second>
__global__ void __launch_bounds__(kBlock)
batch_step2_kernel(const StepParams<T>* __restrict__ descs, const BatchRef* __restrict__ table,
                   const int* __restrict__ ctrl, int step_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BatchRef r = table[blockIdx.x];
  if (r.kind == 3) return;
  const StepParams<T>& p = descs[r.inst];
  const int n = ctrl[0] + step_off;
  if (r.kind == 0) {
    const RowBlock rb = p.blocks[r.idx];
    if constexpr (sizeof(T) == 4) {
      if (rb.kind == 1) {
        coupling_gemm(p, rb, n, reinterpret_cast<float*>(smem));
        return;
      }
    }
    coupling_rows(p, rb, n, reinterpret_cast<T*>(smem));
    return;
  }
  if constexpr (Second) {
    if (r.kind == 1) {
      band_block(p, r.idx / kBandSplit, r.idx % kBandSplit, n);
    } else if (r.kind == 5) {
      switch (p.seg) {
        case 4: stencil2_tile<T, 4, MIdx, true>(p, r.idx, n); break;
        case 16: stencil2_tile<T, 16, MIdx, true>(p, r.idx, n); break;
        case 32: stencil2_tile<T, 32, MIdx, true>(p, r.idx, n); break;
        default: stencil2_tile<T, 8, MIdx, true>(p, r.idx, n); break;
      }
    }
  } else {
    if (r.kind == 1) {
      switch (p.seg) {
        case 4: stencil2_tile<T, 4, MIdx, false>(p, r.idx, n); break;
        case 16: stencil2_tile<T, 16, MIdx, false>(p, r.idx, n); break;
        case 32: stencil2_tile<T, 32, MIdx, false>(p, r.idx, n); break;
        default: stencil2_tile<T, 8, MIdx, false>(p, r.idx, n); break;
      }
      return;
    }
    if (r.kind == 4) {
      switch (p.seg) {
        case 4: stencil2_near<T, 4, MIdx>(p, r.idx, n); break;
        case 16: stencil2_near<T, 16, MIdx>(p, r.idx, n); break;
        case 32: stencil2_near<T, 32, MIdx>(p, r.idx, n); break;
        default: stencil2_near<T, 8, MIdx>(p, r.idx, n); break;
      }
      return;
    }
    pair_probes(p, n);
  }
}

template <typename T>
hipError_t launch_batch_step2(const StepParams<T>* da, const BatchRef* ta, int na, const StepParams<T>* db,
                              const BatchRef* tb, int nb, const int* ctrl, int step_off, size_t smem, bool midx,
                              hipStream_t s) {
  const dim3 blk(kBlock);
  if (midx) {
    hipLaunchKernelGGL((batch_step2_kernel<T, true, false>), dim3(na), blk, smem, s, da, ta, ctrl, step_off);
    if (nb > 0) hipLaunchKernelGGL((batch_step2_kernel<T, true, true>), dim3(nb), blk, smem, s, db, tb, ctrl, step_off + 1);
  } else {
    hipLaunchKernelGGL((batch_step2_kernel<T, false, false>), dim3(na), blk, smem, s, da, ta, ctrl, step_off);
    if (nb > 0) hipLaunchKernelGGL((batch_step2_kernel<T, false, true>), dim3(nb), blk, smem, s, db, tb, ctrl, step_off + 1);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_step(const StepParams<T>* descs, const BatchRef* table, int nblocks,
                             const int* ctrl, int step_off, size_t smem, bool layers, bool midx,
                             hipStream_t s) {
  const dim3 g(nblocks), b(kBlock);
  if (layers && midx)
    hipLaunchKernelGGL((batch_step_kernel<T, true, true>), g, b, smem, s, descs, table, ctrl, step_off);
  else if (layers)
    hipLaunchKernelGGL((batch_step_kernel<T, true, false>), g, b, smem, s, descs, table, ctrl, step_off);
  else if (midx)
    hipLaunchKernelGGL((batch_step_kernel<T, false, true>), g, b, smem, s, descs, table, ctrl, step_off);
  else
    hipLaunchKernelGGL((batch_step_kernel<T, false, false>), g, b, smem, s, descs, table, ctrl, step_off);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_probe_flush(const StepParams<T>* descs, int ninst, const int* ctrl,
                                    int step_off, hipStream_t s) {
  hipLaunchKernelGGL((batch_probe_kernel<T>), dim3(ninst), dim3(kBlock), 0, s, descs, ctrl, step_off);
  return hipGetLastError();
}

// Coarse part of the discrete energy x^T R x of the leap-frog state
// (E^n, Hz^{n-1/2}) (Theorem 2's storage function on the coarse grid): per
// cell its Hz term mu0 dx dy/dt Hz^2 and, for the south Ex and west Ey it
// owns, eps/dt times the edge's dual area (the two half cells that are not
// inside a region; an interface edge keeps its outer half cell, eq. (13))
// times E^2, minus E times the edge's row of K applied to Hz.  One FP64
// partial sum per workgroup.
template <typename T>
__global__ void __launch_bounds__(kBlock)
energy_kernel(const T* __restrict__ hz, const T* __restrict__ ex, const T* __restrict__ ey,
              const T* __restrict__ al, int nx, int ny, int pitch, double ch, double half_area,
              double dx, double dy, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  const int i = blockIdx.x * kWave + (threadIdx.x & (kWave - 1));
  const int j = blockIdx.y * (kBlock / kWave) + threadIdx.x / kWave;
  double e = 0.0;
  if (i < nx && j < ny) {
    const size_t o = (size_t)j * pitch + i;
    const double a = (double)al[o];
    const double h = a > 0 ? (double)hz[o] : 0.0;
    e += ch * h * h;
    if (j >= 1) {
      const double a2 = (double)al[o - pitch];
      const double w = (a > 0 ? a : 0.0) + (a2 > 0 ? a2 : 0.0);
      if (w > 0) {
        const double h2 = a2 > 0 ? (double)hz[o - pitch] : 0.0;
        const double E = (double)ex[o];
        e += half_area * w * E * E - E * dx * (h - h2);
      }
    }
    if (i >= 1) {
      const double a2 = (double)al[o - 1];
      const double w = (a > 0 ? a : 0.0) + (a2 > 0 ? a2 : 0.0);
      if (w > 0) {
        const double h2 = a2 > 0 ? (double)hz[o - 1] : 0.0;
        const double E = (double)ey[o];
        e += half_area * w * E * E - E * dy * (h2 - h);
      }
    }
  }
  for (int off = kWave / 2; off > 0; off >>= 1) e += __shfl_xor(e, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
  }
}

template <typename T>
hipError_t launch_energy(const T* hz, const T* ex, const T* ey, const T* al, int nx, int ny, int pitch,
                         double ch, double half_area, double dx, double dy, double* part, hipStream_t s) {
  const dim3 g((nx + kWave - 1) / kWave, (ny + kBlock / kWave - 1) / (kBlock / kWave));
  hipLaunchKernelGGL((energy_kernel<T>), g, dim3(kBlock), 0, s, hz, ex, ey, al, nx, ny, pitch, ch,
                     half_area, dx, dy, part);
  return hipGetLastError();
}

template hipError_t launch_energy<float>(const float*, const float*, const float*, const float*, int, int,
                                         int, double, double, double, double, double*, hipStream_t);
template hipError_t launch_energy<double>(const double*, const double*, const double*, const double*, int,
                                          int, int, double, double, double, double, double*, hipStream_t);

template <typename T>
hipError_t launch_step(const StepParams<T>& p, int seg, size_t smem, hipStream_t s) {
  const dim3 g(p.ncoup_blocks + p.nst_blocks + 1), b(kBlock);
  // kernel variant: tile height, absorbing layers present, material table
  auto go = [&](auto layers, auto midx) -> hipError_t {
    constexpr bool Lf = decltype(layers)::value, Mf = decltype(midx)::value;
    switch (seg) {
      case 4: hipLaunchKernelGGL((step_kernel<T, 4, Lf, Mf>), g, b, smem, s, p); break;
      case 8: hipLaunchKernelGGL((step_kernel<T, 8, Lf, Mf>), g, b, smem, s, p); break;
      case 16: hipLaunchKernelGGL((step_kernel<T, 16, Lf, Mf>), g, b, smem, s, p); break;
      case 32: hipLaunchKernelGGL((step_kernel<T, 32, Lf, Mf>), g, b, smem, s, p); break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  };
  using Y = std::true_type;
  using N = std::false_type;
  const hipError_t e = p.pml ? (p.midx ? go(Y{}, Y{}) : go(Y{}, N{})) : (p.midx ? go(N{}, Y{}) : go(N{}, N{}));
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step2(const StepParams<T>& a, const StepParams<T>& b, int seg, size_t smem, hipStream_t s) {
  // the second launch has nothing to do without regions and with every far
  // tile in the first
  const int nn = a.n_near * (seg / std::min(a.near_rows, seg));
  const dim3 ga(a.ncoup_blocks + ((nn + 7) & ~7) + a.far_split + 1),
      gb(b.ncoup_blocks + ((b.n_band * kBandSplit + 7) & ~7) + (b.nst2_blocks - b.far_split)), blk(kBlock);
  auto go = [&](auto midx) -> hipError_t {
    constexpr bool Mf = decltype(midx)::value;
    switch (seg) {
      case 4:
        hipLaunchKernelGGL((step2_kernel<T, 4, Mf, false>), ga, blk, smem, s, a);
        if (gb.x > 0) hipLaunchKernelGGL((step2_kernel<T, 4, Mf, true>), gb, blk, smem, s, b);
        break;
      case 8:
        hipLaunchKernelGGL((step2_kernel<T, 8, Mf, false>), ga, blk, smem, s, a);
        if (gb.x > 0) hipLaunchKernelGGL((step2_kernel<T, 8, Mf, true>), gb, blk, smem, s, b);
        break;
      case 16:
        hipLaunchKernelGGL((step2_kernel<T, 16, Mf, false>), ga, blk, smem, s, a);
        if (gb.x > 0) hipLaunchKernelGGL((step2_kernel<T, 16, Mf, true>), gb, blk, smem, s, b);
        break;
      case 32:
        hipLaunchKernelGGL((step2_kernel<T, 32, Mf, false>), ga, blk, smem, s, a);
        if (gb.x > 0) hipLaunchKernelGGL((step2_kernel<T, 32, Mf, true>), gb, blk, smem, s, b);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  };
  const hipError_t e = a.midx ? go(std::true_type{}) : go(std::false_type{});
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_probe_flush(const StepParams<T>& p, hipStream_t s) {
  hipLaunchKernelGGL((probe_kernel<T>), dim3(1), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_tick(int* ctrl, int k, hipStream_t s) {
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, s, ctrl, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_finite_check(const T* f, size_t n, int* flag, hipStream_t s) {
  if (n % (16 / sizeof(T)) != 0 || ((uintptr_t)f) % 16 != 0) return hipErrorInvalidValue;
  const size_t nv = n / (16 / sizeof(T));
  const size_t want = (nv + kBlock - 1) / kBlock;
  const unsigned g = (unsigned)std::max<size_t>(1, std::min<size_t>(want, 2048));
  hipLaunchKernelGGL((finite_check_kernel<T>), dim3(g), dim3(kBlock), 0, s, f, n, flag);
  return hipGetLastError();
}
template hipError_t launch_finite_check<float>(const float*, size_t, int*, hipStream_t);
template hipError_t launch_finite_check<double>(const double*, size_t, int*, hipStream_t);

template hipError_t launch_step<float>(const StepParams<float>&, int, size_t, hipStream_t);
template hipError_t launch_step<double>(const StepParams<double>&, int, size_t, hipStream_t);
template hipError_t launch_step2<float>(const StepParams<float>&, const StepParams<float>&, int, size_t, hipStream_t);
template hipError_t launch_step2<double>(const StepParams<double>&, const StepParams<double>&, int, size_t, hipStream_t);
template hipError_t launch_probe_flush<float>(const StepParams<float>&, hipStream_t);
template hipError_t launch_probe_flush<double>(const StepParams<double>&, hipStream_t);
template hipError_t launch_batch_step<float>(const StepParams<float>*, const BatchRef*, int, const int*,
                                             int, size_t, bool, bool, hipStream_t);
template hipError_t launch_batch_step<double>(const StepParams<double>*, const BatchRef*, int,
                                              const int*, int, size_t, bool, bool, hipStream_t);
template hipError_t launch_batch_step2<float>(const StepParams<float>*, const BatchRef*, int, const StepParams<float>*,
                                              const BatchRef*, int, const int*, int, size_t, bool, hipStream_t);
template hipError_t launch_batch_step2<double>(const StepParams<double>*, const BatchRef*, int,
                                               const StepParams<double>*, const BatchRef*, int, const int*, int,
                                               size_t, bool, hipStream_t);
template hipError_t launch_batch_probe_flush<float>(const StepParams<float>*, int, const int*, int,
                                                    hipStream_t);
template hipError_t launch_batch_probe_flush<double>(const StepParams<double>*, int, const int*, int,
                                                     hipStream_t);

}  // namespace fdtd
