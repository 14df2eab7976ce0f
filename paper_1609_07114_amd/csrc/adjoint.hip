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
#include "adjoint.hpp"
#include "device.hpp"

namespace fdtd {

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

// One lane's column of row j for the reverse sweep.
template <typename T>
struct AdjRow {
  T a, b, h;      // material (a < 0 inside regions, 0 in padding), forward Hz^{n+1/2}
  T lx, e;        // adjoint and forward value of the row's south Ex
  T lh, ly, ey;   // adjoint Hz, adjoint and forward value of the west Ey
};

// Loads are unconditional from a valid offset (`ob` when `ok`, else cell
// (0,0)) and the values of lanes without data are selected to zero: no
// lane-divergent branches.
template <typename T>
__device__ __forceinline__ AdjRow<T> adj_load(const AdjParams<T>& p, uint32_t ob, bool ok) {
  const uint32_t o = ok ? ob : 0u;
  AdjRow<T> r;
  r.a = ld(p.al, o);
  r.b = ld(p.be, o);
  r.h = ld(p.hz1, o);
  r.lx = ld(p.lex_in, o);
  r.e = ld(p.ex0, o);
  r.lh = ld(p.lhz_in, o);
  r.ly = ld(p.ley_in, o);
  r.ey = ld(p.ey0, o);
  if (!ok) r = AdjRow<T>{T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  return r;
}

constexpr int kAdjOwned = kWave - 3;  // columns a reverse-sweep wave owns

// Transposed eq. (3) + eq. (5) and the coefficient gradients, streamed up
// the rows like the forward stencil.  A wave covers 64 lanes = columns
// iw-2 .. iw+61 (iw = 61 * blockIdx.x).  Lanes 2..62 own their column; lane 1
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
template <typename T, int SEG>
__global__ void __launch_bounds__(kBlock) adj_stream(const AdjParams<T> p) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int iw = blockIdx.x * kAdjOwned;
  const int ic = iw - 2 + lane;
  const int j0 = (blockIdx.y * (kBlock / kWave) + wv) * SEG;
  if (j0 >= p.ny) return;
  const int j1 = min(j0 + SEG, p.ny);
  const int js = j0 > 0 ? j0 - 1 : 0;
  const int nx = p.nx, ny = p.ny;
  constexpr uint32_t ts = sizeof(T);
  const uint32_t row_b = (uint32_t)p.pitch * ts;
  const bool in = ic >= 0 && ic < nx;
  const bool own = in && lane >= 2 && lane <= kWave - 2;
  const T chdy = p.chdy, chdx = p.chdx, k2dy = p.k2dy, k2dx = p.k2dx;
  const T idx = T(1.0 / p.dx), idy = T(1.0 / p.dy);  // reciprocal lengths
  const double fa = p.fa;
  // byte offset of (ic, js); only dereferenced where `in`
  uint32_t ob = ((uint32_t)js * (uint32_t)p.pitch + (uint32_t)ic) * ts;
  const uint32_t obj_b = (uint32_t)(p.obj_off * ts);
  // byte offset of the same cell in the FP64 accumulators
  auto o8 = [](uint32_t obt) -> uint32_t { return obt / ts * 8u; };

  AdjRow<T> prv = adj_load(p, ob - row_b, in && js >= 1);
  AdjRow<T> cur = adj_load(p, ob, in);
  AdjRow<T> nxt = adj_load(p, ob + row_b, in && js + 1 < ny);
  T mu_p = T(0);
  T gpa = T(0), gpb = T(0);             // previous row's cell: dJ/da, dJ/db of all edges but its north
  double acc_e = 0.0, acc_s = 0.0;      // its accumulators, read one row ahead
  T cas = T(0), cbs = T(0), rs = T(0);  // current row's south edge
  adj_coef(cur.a + prv.a, cur.b + prv.b, k2dy, cas, cbs, rs);
#pragma unroll
  for (int it = 0; it <= SEG; ++it) {
    const int j = js + it;
    if (j >= j1) break;
    const bool up = j + 1 < ny;
    // row j+2 in flight (needed as the north row of the next iteration)
    const bool up2 = j + 2 < ny && j + 1 < j1;
    const AdjRow<T> nn = adj_load(p, ob + 2 * row_b, in && up2);
    // this row's accumulators (this wave is their only writer), stored next row
    const bool acc_row = j >= j0 && own;
    double nacc_e = ld(p.geps, acc_row ? o8(ob) : 0u);
    double nacc_s = ld(p.gsig, acc_row ? o8(ob) : 0u);
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
    T mu = cur.lh;
    mu += (in && ob == obj_b) ? p.obj_coef * cur.h : T(0);
    mu += actS ? cbs * cur.lx : T(0);
    mu -= actN ? cbn * nxt.lx : T(0);
    mu -= actW ? cbw * cur.ly : T(0);
    mu += actE ? cbe * lye : T(0);
    mu = act ? mu : T(0);
    const T mu_w = lane_prev(mu);
    // gradient shares of the south, west and east edges
    T gas = T(0), gbs = T(0), gaw = T(0), gbw = T(0), gae = T(0), gbe = T(0);
    edge_grad(cur.lx, cur.e, cur.h - prv.h, cur.a + prv.a, cur.b + prv.b, rs, idy, gas, gbs);
    edge_grad(cur.ly, cur.ey, -(cur.h - hw), cur.a + aw, cur.b + bw, rw, idx, gaw, gbw);
    edge_grad(lye, eye, -(he - cur.h), ae + cur.a, be_ + cur.b, re, idx, gae, gbe);
    gas = actS ? gas : T(0);
    gbs = actS ? gbs : T(0);
    gaw = actW ? gaw : T(0);
    gbw = actW ? gbw : T(0);
    gae = actE ? gae : T(0);
    gbe = actE ? gbe : T(0);
    if (acc_row) {
      const T lxo = chdy * (mu_p - mu) + (actS ? cas * cur.lx : T(0));
      const T lyo = chdx * (mu - mu_w) + (actW ? caw * cur.ly : T(0));
      st(p.lhz_out, ob, mu);
      st(p.lex_out, ob, j >= 1 ? lxo : T(0));
      st(p.ley_out, ob, ic >= 1 ? lyo : T(0));
      // the previous row's cell is complete with its north edge (= this row's south)
      if (j - 1 >= j0) {
        st(p.geps, o8(ob - row_b), acc_e + fa * (double)(gpa + gas));
        st(p.gsig, o8(ob - row_b), acc_s + 0.25 * (double)(gpb + gbs));
      }
    }
    gpa = gas + gaw + gae;
    gpb = gbs + gbw + gbe;
    acc_e = nacc_e;
    acc_s = nacc_s;
    mu_p = mu;
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
    const uint32_t oc = o8(ob - row_b);
    T gna = T(0), gnb = T(0);
    if (j1 < ny && prv.a > T(0) && cur.a > T(0))
      edge_grad(cur.lx, cur.e, cur.h - prv.h, cur.a + prv.a, cur.b + prv.b, rs, idy, gna, gnb);
    st(p.geps, oc, acc_e + fa * (double)(gpa + gna));
    st(p.gsig, oc, acc_s + 0.25 * (double)(gpb + gnb));
  }
}

template <typename T>
hipError_t launch_adjoint_step(const AdjParams<T>& p, size_t smem, hipStream_t s) {
  if (p.nblocks > 0) hipLaunchKernelGGL((adj_coupling<T>), dim3(p.nblocks), dim3(kBlock), smem, s, p);
  const int rows = (kBlock / kWave) * p.seg;
  const dim3 g((p.nx + kAdjOwned - 1) / kAdjOwned, (p.ny + rows - 1) / rows);
  switch (p.seg) {
    case 4: hipLaunchKernelGGL((adj_stream<T, 4>), g, dim3(kBlock), 0, s, p); break;
    case 8: hipLaunchKernelGGL((adj_stream<T, 8>), g, dim3(kBlock), 0, s, p); break;
    case 16: hipLaunchKernelGGL((adj_stream<T, 16>), g, dim3(kBlock), 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const AdjParams<float>&, size_t, hipStream_t);
template hipError_t launch_adjoint_step<double>(const AdjParams<double>&, size_t, hipStream_t);

}  // namespace fdtd
