// Batched runs (fdtd_rom_batch_*): B independent problems, each laid out by
// the single-problem path in its own slice of one device workspace, advanced
// together by one launch per step (batch_step_kernel) whose workgroups walk
// a table of (instance, role, index).  Table order: every instance's coupling
// blocks first (the longest workgroups start first), then each instance's
// stencil tiles from an index that is a multiple of 8 (so the XCD-aware tile
// remap of the single-problem kernel holds per instance), then one probe
// block per instance.  run() replays captured graphs of `graph_batch` steps.
//
// Two steps per pass (the default when no instance has absorbing layers):
// steps go in pairs of launches of batch_step2_kernel over two more tables
// (first launch: coupling blocks, every instance's two-step tiles, probe
// blocks; second: coupling blocks, every instance's band blocks, one per
// region).  All instances step in lockstep, so one parity and one set-order
// bit describe them all; the descriptors of both set orders (single-step,
// first and second launch) are uploaded for the parity the pairs start at.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fdtd_rom.h"
#include "runtime.hpp"

using namespace fdtd;

struct fdtd_rom_batch {
  int dtype = FDTD_F32;
  int B = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  std::vector<fdtd_rom_sim*> sims;
  size_t off_ctrl = 0, off_desc = 0, off_table = 0;
  size_t table_cap = 0;
  std::vector<BatchRef> table;
  // two steps per pass: tables of the pair's launches, descriptor sets
  // [single, first, second] x [set order 0, 1] (each B entries)
  bool tb = false;
  int tb_key = -1;       // (parity the pairs start at) | set order << 1 at the last upload
  int graph_key = -1;
  size_t off_tab2a = 0, off_tab2b = 0, tab2_cap = 0, desc_stride = 0;
  std::vector<BatchRef> tab2a, tab2b;
  size_t smem = 0;
  bool layers = false;  // some instance has absorbing layers: launch the kernel variant with them
  bool midx = false;    // every instance reads its material from a table
  bool dirty = true;  // descriptors / table must be uploaded before the next launch
  int steps = 0;
  int graph_batch = 0;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
};

namespace {

int tiles_for(const fdtd_problem& p, int seg) {
  const int rows = (kBlock / kWave) * seg;
  return ((p.grid.nx + kWave - 1) / kWave) * ((p.grid.ny + rows - 1) / rows);
}

struct BatchPlan {
  std::vector<size_t> inst_off, inst_bytes;
  size_t off_ctrl = 0, off_desc = 0, off_table = 0, table_cap = 0, total = 0;
  size_t off_tab2a = 0, off_tab2b = 0, tab2_cap = 0, desc_stride = 0;
};

int plan_batch(const fdtd_problem* probs, int B, BatchPlan& P) {
  if (!probs || B < 1) return fail(FDTD_EINVAL, "need at least one instance");
  const int dt = probs[0].grid.dtype;
  size_t cap = 8, cap2 = 8;
  P.inst_off.assign(B, 0);
  P.inst_bytes.assign(B, 0);
  std::vector<size_t> sizes(B);
  for (int b = 0; b < B; ++b) {
    if (probs[b].grid.dtype != dt) return fail(FDTD_EINVAL, "instance %d: every instance must share one dtype", b);
    Layout L;
    const int rc = plan_problem(&probs[b], L);
    if (rc != FDTD_OK) return fail(rc, "instance %d: %s", b, fdtd_rom_last_error());
    sizes[b] = L.total;
    cap += (size_t)std::max(L.nrowblocks, L.nblocks_mixed) + (size_t)tiles_for(probs[b], 4) + 14 + 1;
    // first table: coupling blocks, near-tile pieces (at most twice the
    // tile count of 4-row waves: a near tile of SEG-row waves is SEG/2
    // pieces), tiles, two paddings, probe block; second: coupling and band
    cap2 += (size_t)std::max(L.nrowblocks, L.nblocks_mixed) +
            std::max((size_t)L.max_tiles2 * 3 + 16, (size_t)L.max_tiles2 + (size_t)probs[b].nroms * kBandSplit) + 21 + 1;
  }
  const size_t desc_bytes = (size_t)B * (dt == FDTD_F32 ? sizeof(StepParams<float>) : sizeof(StepParams<double>));
  P.desc_stride = align_up(desc_bytes, 256);
  size_t o = 0;
  P.off_ctrl = o;
  o = align_up(o + kCtrlInts * sizeof(int), 256);
  P.off_desc = o;
  o += 6 * P.desc_stride;
  P.off_table = o;
  P.table_cap = cap;
  o = align_up(o + cap * sizeof(BatchRef), 256);
  P.tab2_cap = cap2;
  P.off_tab2a = o;
  o = align_up(o + cap2 * sizeof(BatchRef), 256);
  P.off_tab2b = o;
  o = align_up(o + cap2 * sizeof(BatchRef), 256);
  for (int b = 0; b < B; ++b) {
    P.inst_off[b] = o;
    P.inst_bytes[b] = sizes[b];
    o = align_up(o + sizes[b], 256);
  }
  P.total = o;
  return FDTD_OK;
}

void build_table(fdtd_rom_batch* bt) {
  std::vector<BatchRef>& t = bt->table;
  t.clear();
  auto pad8 = [&]() {
    while (t.size() % 8) t.push_back(BatchRef{0, 3, 0, 0});
  };
  // the parameter block of the handle's own dtype (the other stays unset)
  auto nrow = [&](int b) { return bt->dtype == FDTD_F32 ? bt->sims[b]->sp_f.nrowblocks : bt->sims[b]->sp_d.nrowblocks; };
  auto ntile = [&](int b) { return bt->dtype == FDTD_F32 ? bt->sims[b]->sp_f.nst_blocks : bt->sims[b]->sp_d.nst_blocks; };
  // each instance's coupling blocks from an index that is a multiple of 8,
  // so that the handle's XCD grouping of a model's blocks holds
  for (int b = 0; b < bt->B; ++b) {
    pad8();
    for (int k = 0; k < nrow(b); ++k) t.push_back(BatchRef{b, 0, k, 0});
  }
  for (int b = 0; b < bt->B; ++b) {
    pad8();
    for (int k = 0; k < ntile(b); ++k) t.push_back(BatchRef{b, 1, k, 0});
  }
  for (int b = 0; b < bt->B; ++b) t.push_back(BatchRef{b, 2, 0, 0});
  if (bt->tb) {
    auto two = [&](std::vector<BatchRef>& u, bool second) {
      u.clear();
      for (int b = 0; b < bt->B; ++b) {
        while (u.size() % 8) u.push_back(BatchRef{0, 3, 0, 0});
        for (int k = 0; k < nrow(b); ++k) u.push_back(BatchRef{b, 0, k, 0});
      }
      for (int b = 0; b < bt->B; ++b) {
        while (u.size() % 8) u.push_back(BatchRef{0, 3, 0, 0});
        const fdtd_rom_sim* sb = bt->sims[b];
        // first launch: the instance's near-tile pieces, then its two-step
        // tiles (the near ones return at once); second: its band blocks
        // (one per region)
        const int n_near = bt->dtype == FDTD_F32 ? sb->sp_f.n_near : sb->sp_d.n_near;
        const int near_rows = bt->dtype == FDTD_F32 ? sb->sp_f.near_rows : sb->sp_d.near_rows;
        const int nt = bt->dtype == FDTD_F32 ? sb->sp_f.nst2_blocks : sb->sp_d.nst2_blocks;
        const int split = bt->dtype == FDTD_F32 ? sb->sp_f.far_split : sb->sp_d.far_split;
        // near pieces and band blocks are listed in the order the single
        // handle's launch remaps them to (each XCD a contiguous run, so a
        // region's pieces share an L2); entries start at a multiple of 8,
        // so entry k runs on XCD k % 8
        auto xcd_order = [&](int cnt, int kind) {
          const int cnt8 = (cnt + 7) & ~7, per = cnt8 / 8;
          for (int k = 0; k < cnt8; ++k) {
            const int v = (k & 7) * per + (k >> 3);
            u.push_back(v < cnt ? BatchRef{b, kind, v, 0} : BatchRef{0, 3, 0, 0});
          }
        };
        if (second) {
          xcd_order(sb->nroms * kBandSplit, 1);
          for (int k = 0; k < nt - split; ++k) u.push_back(BatchRef{b, 5, k, 0});
        } else {
          const int nn = n_near * (sb->seg / std::min(near_rows, sb->seg));
          xcd_order(nn, 4);
          for (int k = 0; k < split; ++k) u.push_back(BatchRef{b, 1, k, 0});
        }
      }
      if (!second)
        for (int b = 0; b < bt->B; ++b) u.push_back(BatchRef{b, 2, 0, 0});
    };
    two(bt->tab2a, false);
    two(bt->tab2b, true);
  }
  bt->smem = 0;
  bt->layers = false;
  bt->midx = true;
  for (int b = 0; b < bt->B; ++b) {
    const fdtd_rom_sim* sb = bt->sims[b];
    bt->smem = std::max(bt->smem, sb->smem);
    bt->layers = bt->layers || sb->L.pml;
    bt->midx = bt->midx && (bt->dtype == FDTD_F32 ? sb->sp_f.midx : sb->sp_d.midx) != 0;
  }
}

void drop_batch_graph(fdtd_rom_batch* bt) {
  if (bt->graph) (void)hipGraphExecDestroy(bt->graph);
  bt->graph = nullptr;
  bt->graph_steps = 0;
}

template <typename T>
int upload(fdtd_rom_batch* bt) {
  if (bt->tb)
    for (fdtd_rom_sim* s : bt->sims) {
      const int rc = prepare_tb<T>(s);
      if (rc != FDTD_OK) return rc;
    }
  build_table(bt);
  if (bt->table.size() > bt->table_cap) return fail(FDTD_EINVAL, "internal: batch table overflow");
  if (bt->tb && (bt->tab2a.size() > bt->tab2_cap || bt->tab2b.size() > bt->tab2_cap))
    return fail(FDTD_EINVAL, "internal: batch pair table overflow");
  // descriptor sets [single, first, second] for set order 0 and 1, the
  // pairs starting at parity par; the handles' own parameters hold the
  // current order
  const int flip = bt->sims[0]->flip;
  const int par = bt->steps & 1;
  std::vector<StepParams<T>> d(6 * (size_t)bt->B);
  for (int b = 0; b < bt->B; ++b) {
    fdtd_rom_sim* s = bt->sims[b];
    for (int o = 0; o < 2; ++o) {
      StepParams<T> sp = step_params<T>(s);
      if (o != flip)
        for (int c = 0; c < 3; ++c) std::swap(sp.f[0][c], sp.f[1][c]);
      d[(size_t)(3 * o) * bt->B + b] = sp;
      if (!bt->tb) continue;
      T* fc[3];
      for (int c = 0; c < 3; ++c) fc[c] = (T*)(s->ws + s->L.off_fc + c * s->L.field_elems * sizeof(T));
      StepParams<T> a = sp, b2 = sp;
      for (int c = 0; c < 3; ++c) {
        a.f[par ^ 1][c] = fc[c];
        a.f2[c] = sp.f[par ^ 1][c];
        b2.f[par ^ 1][c] = fc[c];
        b2.f[par][c] = sp.f[par ^ 1][c];
        b2.f2[c] = sp.f[par][c];  // the second launch's far tiles read step n
      }
      d[(size_t)(3 * o + 1) * bt->B + b] = a;
      d[(size_t)(3 * o + 2) * bt->B + b] = b2;
    }
  }
  for (int k = 0; k < 6; ++k)
    if (hipMemcpyAsync(bt->ws + bt->off_desc + k * bt->desc_stride, d.data() + (size_t)k * bt->B,
                       bt->B * sizeof(StepParams<T>), hipMemcpyHostToDevice, bt->stream) != hipSuccess)
      return fail(FDTD_EDEVICE, "batch descriptor upload failed");
  if (hipMemcpyAsync(bt->ws + bt->off_table, bt->table.data(), bt->table.size() * sizeof(BatchRef),
                     hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
      (bt->tb && (hipMemcpyAsync(bt->ws + bt->off_tab2a, bt->tab2a.data(), bt->tab2a.size() * sizeof(BatchRef),
                                 hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
                  hipMemcpyAsync(bt->ws + bt->off_tab2b, bt->tab2b.data(), bt->tab2b.size() * sizeof(BatchRef),
                                 hipMemcpyHostToDevice, bt->stream) != hipSuccess)) ||
      hipStreamSynchronize(bt->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "batch descriptor upload failed");
  bt->tb_key = par | (flip << 1);
  bt->dirty = false;
  return FDTD_OK;
}

// the handles' current set order after the pairs of a run
template <typename T>
void flip_sets(fdtd_rom_batch* bt) {
  for (fdtd_rom_sim* s : bt->sims) {
    StepParams<T>& sp = step_params<T>(s);
    for (int c = 0; c < 3; ++c) std::swap(sp.f[0][c], sp.f[1][c]);
    s->flip ^= 1;
  }
}

// Enqueue nsteps steps (pairs first when two steps per pass are on, then a
// last odd step), the probe flush and the tick; *pairs receives the number
// of pairs (each trades the two field sets' places).
template <typename T>
int enqueue_batch(fdtd_rom_batch* bt, int nsteps, hipStream_t st, int* pairs) {
  auto desc = [&](int o, int k) { return (const StepParams<T>*)(bt->ws + bt->off_desc + (3 * o + k) * bt->desc_stride); };
  const BatchRef* tab = (const BatchRef*)(bt->ws + bt->off_table);
  int* ctrl = (int*)(bt->ws + bt->off_ctrl);
  int o = bt->sims[0]->flip;
  int k = 0;
  *pairs = 0;
  if (bt->tb) {
    const BatchRef* ta = (const BatchRef*)(bt->ws + bt->off_tab2a);
    const BatchRef* tb2 = (const BatchRef*)(bt->ws + bt->off_tab2b);
    for (; k + 2 <= nsteps; k += 2) {
      if (launch_batch_step2<T>(desc(o, 1), ta, (int)bt->tab2a.size(), desc(o, 2), tb2, (int)bt->tab2b.size(), ctrl, k,
                                bt->smem, bt->midx, st) != hipSuccess)
        return fail(FDTD_EDEVICE, "batch pair launch failed: %s", hipGetErrorString(hipGetLastError()));
      o ^= 1;
      ++*pairs;
    }
  }
  for (; k < nsteps; ++k)
    if (launch_batch_step<T>(desc(o, 0), tab, (int)bt->table.size(), ctrl, k, bt->smem, bt->layers, bt->midx, st) !=
        hipSuccess)
      return fail(FDTD_EDEVICE, "batch step launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (launch_batch_probe_flush<T>(desc(o, 0), bt->B, ctrl, nsteps, st) != hipSuccess ||
      launch_tick(ctrl, nsteps, st) != hipSuccess)
    return fail(FDTD_EDEVICE, "batch probe/tick launch failed");
  return FDTD_OK;
}

template <typename T>
int capture_batch(fdtd_rom_batch* bt, int gb) {
  drop_batch_graph(bt);
  if (!bt->cap_stream && hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamCreateWithFlags failed");
  if (hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamBeginCapture failed");
  int pairs = 0;
  int rc = enqueue_batch<T>(bt, gb, bt->cap_stream, &pairs);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(bt->cap_stream, &g);
  if (rc == FDTD_OK && (pairs & 1)) rc = fail(FDTD_EINVAL, "internal: odd pair count in a captured batch");
  if (rc != FDTD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess || !g) return fail(FDTD_EDEVICE, "hipStreamEndCapture failed");
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return fail(FDTD_EDEVICE, "hipGraphInstantiate failed");
  bt->graph = ex;
  bt->graph_steps = gb;
  bt->graph_key = bt->tb_key;
  return FDTD_OK;
}

// Captured batches hold fixed descriptor and table addresses; with two
// steps per pass they are a multiple of 4 steps (an even number of pairs:
// parity and set order unchanged) and are keyed on the parity and set order
// their descriptors were uploaded for.
template <typename T>
int run_batch(fdtd_rom_batch* bt, int nsteps) {
  const int key = (bt->steps & 1) | (bt->sims[0]->flip << 1);
  if (bt->dirty || (bt->tb && bt->tb_key != key)) {
    if (bt->dirty) drop_batch_graph(bt);  // tables may have changed size
    const int rc = upload<T>(bt);
    if (rc != FDTD_OK) return rc;
  }
  int done = 0;
  const int gb = bt->tb ? bt->graph_batch / 4 * 4 : bt->graph_batch;
  if (gb > 0 && nsteps >= gb) {
    if (!bt->graph || bt->graph_steps != gb || bt->graph_key != bt->tb_key) {
      const int rc = capture_batch<T>(bt, gb);
      if (rc != FDTD_OK) return rc;
    }
    while (nsteps - done >= gb) {
      if (hipGraphLaunch(bt->graph, bt->stream) != hipSuccess)
        return fail(FDTD_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(hipGetLastError()));
      done += gb;
    }
  }
  if (nsteps > done) {
    int pairs = 0;
    const int rc = enqueue_batch<T>(bt, nsteps - done, bt->stream, &pairs);
    if (rc != FDTD_OK) return rc;
    if (pairs & 1) flip_sets<T>(bt);
  }
  for (fdtd_rom_sim* s : bt->sims) s->steps += nsteps;
  bt->steps += nsteps;
  return FDTD_OK;
}

}  // namespace

extern "C" {

int fdtd_rom_batch_workspace_size(const fdtd_problem* probs, int32_t B, size_t* bytes) {
  if (!bytes) return fail(FDTD_EINVAL, "null output");
  try {
    BatchPlan P;
    const int rc = plan_batch(probs, B, P);
    if (rc != FDTD_OK) return rc;
    *bytes = P.total;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_batch_create(const fdtd_problem* probs, int32_t B, void* dev_workspace, size_t ws_bytes,
                          void* hip_stream, fdtd_rom_batch** out) {
  if (!out) return fail(FDTD_EINVAL, "null output handle");
  *out = nullptr;
  try {
    BatchPlan P;
    int rc = plan_batch(probs, B, P);
    if (rc != FDTD_OK) return rc;
    if (!dev_workspace) return fail(FDTD_EINVAL, "null workspace");
    if (((uintptr_t)dev_workspace) % 256) return fail(FDTD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < P.total) return fail(FDTD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, P.total);
    fdtd_rom_batch* bt = new fdtd_rom_batch();
    bt->dtype = probs[0].grid.dtype;
    bt->B = B;
    bt->stream = (hipStream_t)hip_stream;
    bt->ws = (char*)dev_workspace;
    bt->off_ctrl = P.off_ctrl;
    bt->off_desc = P.off_desc;
    bt->off_table = P.off_table;
    bt->table_cap = P.table_cap;
    bt->off_tab2a = P.off_tab2a;
    bt->off_tab2b = P.off_tab2b;
    bt->tab2_cap = P.tab2_cap;
    bt->desc_stride = P.desc_stride;
    for (int b = 0; b < B && rc == FDTD_OK; ++b) {
      fdtd_rom_sim* s = nullptr;
      rc = fdtd_rom_create(&probs[b], bt->ws + P.inst_off[b], P.inst_bytes[b], hip_stream, &s);
      if (rc != FDTD_OK) {
        rc = fail(rc, "instance %d: %s", b, fdtd_rom_last_error());
        break;
      }
      // the batch launches every instance itself; its handle never runs
      s->tb = false;
      bt->sims.push_back(s);
    }
    if (rc == FDTD_OK) {
      // two steps per pass when no instance has absorbing layers
      bt->tb = true;
      for (fdtd_rom_sim* s : bt->sims) bt->tb = bt->tb && s->L.tb_ok;
      for (fdtd_rom_sim* s : bt->sims)
        set_tiling(s, bt->tb ? default_tiling2(s->nx, s->ny, (int)s->L.tsize) : default_tiling(s->nx, s->ny, (int)s->L.tsize));
    }
    int ctrl[kCtrlInts] = {0, 0, 0, 0};
    if (rc == FDTD_OK &&
        (hipMemcpyAsync(bt->ws + bt->off_ctrl, ctrl, sizeof(ctrl), hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
         hipStreamSynchronize(bt->stream) != hipSuccess))
      rc = fail(FDTD_EDEVICE, "hipMemcpyAsync failed");
    if (rc == FDTD_OK) rc = bt->dtype == FDTD_F32 ? upload<float>(bt) : upload<double>(bt);
    if (rc != FDTD_OK) {
      fdtd_rom_batch_destroy(bt);
      return rc;
    }
    *out = bt;
    return FDTD_OK;
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_batch_run(fdtd_rom_batch* bt, int32_t nsteps) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (nsteps < 0) return fail(FDTD_EINVAL, "negative step count");
  if (nsteps == 0) return FDTD_OK;
  for (int b = 0; b < bt->B; ++b)
    if ((int64_t)bt->sims[b]->steps + nsteps > bt->sims[b]->max_steps)
      return fail(FDTD_ESTATE, "instance %d: %d + %d steps exceed max_steps=%d", b, bt->sims[b]->steps, nsteps,
                  bt->sims[b]->max_steps);
  try {
    return bt->dtype == FDTD_F32 ? run_batch<float>(bt, nsteps) : run_batch<double>(bt, nsteps);
  } catch (const std::bad_alloc&) {
    return fail(FDTD_ENOMEM, "host allocation failed");
  }
}

int fdtd_rom_batch_steps_done(const fdtd_rom_batch* bt, int32_t* n) {
  if (!bt || !n) return fail(FDTD_EINVAL, "null argument");
  *n = bt->steps;
  return FDTD_OK;
}

int fdtd_rom_batch_read_probes(const fdtd_rom_batch* bt, int32_t b, int32_t first, int32_t count,
                               double* host_out) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (b < 0 || b >= bt->B) return fail(FDTD_EINVAL, "instance %d out of range", b);
  return fdtd_rom_read_probes(bt->sims[b], first, count, host_out);
}

int fdtd_rom_batch_read_field(const fdtd_rom_batch* bt, int32_t b, int32_t comp, double* host_out) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (b < 0 || b >= bt->B) return fail(FDTD_EINVAL, "instance %d out of range", b);
  return fdtd_rom_read_field(bt->sims[b], comp, host_out);
}

int fdtd_rom_batch_set_tiling(fdtd_rom_batch* bt, int32_t b, int32_t seg) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (b < -1 || b >= bt->B) return fail(FDTD_EINVAL, "instance %d out of range", b);
  if (seg != 4 && seg != 8 && seg != 16 && seg != 32) return fail(FDTD_EINVAL, "segment rows must be 4, 8, 16 or 32");
  for (int k = 0; k < bt->B; ++k)
    if (b < 0 || k == b) set_tiling(bt->sims[k], seg);
  bt->dirty = true;
  return FDTD_OK;
}

int fdtd_rom_batch_set_pair_split(fdtd_rom_batch* bt, int32_t b, int32_t percent) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (b < -1 || b >= bt->B) return fail(FDTD_EINVAL, "instance %d out of range", b);
  for (int k = 0; k < bt->B; ++k)
    if (b < 0 || k == b) {
      const int rc = fdtd_rom_set_pair_split(bt->sims[k], percent);
      if (rc != FDTD_OK) return rc;
    }
  drop_batch_graph(bt);  // the pair tables change size
  bt->dirty = true;
  return FDTD_OK;
}

int fdtd_rom_batch_set_time_blocking(fdtd_rom_batch* bt, int32_t on) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (on != 0 && on != 1) return fail(FDTD_EINVAL, "time blocking must be 0 or 1");
  if (on)
    for (int b = 0; b < bt->B; ++b)
      if (!bt->sims[b]->L.tb_ok) return fail(FDTD_EINVAL, "instance %d has absorbing layers: no two-step launches", b);
  bt->tb = on != 0;
  drop_batch_graph(bt);
  bt->dirty = true;
  return FDTD_OK;
}

int fdtd_rom_batch_get_time_blocking(const fdtd_rom_batch* bt, int32_t* on) {
  if (!bt || !on) return fail(FDTD_EINVAL, "null argument");
  *on = bt->tb ? 1 : 0;
  return FDTD_OK;
}

int fdtd_rom_batch_set_graph(fdtd_rom_batch* bt, int32_t batch) {
  if (!bt) return fail(FDTD_EINVAL, "null handle");
  if (batch < 0 || batch > 4096) return fail(FDTD_EINVAL, "graph batch must be in [0, 4096]");
  bt->graph_batch = batch;
  drop_batch_graph(bt);
  return FDTD_OK;
}

void fdtd_rom_batch_destroy(fdtd_rom_batch* bt) {
  if (!bt) return;
  (void)hipStreamSynchronize(bt->stream);
  drop_batch_graph(bt);
  if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
  for (fdtd_rom_sim* s : bt->sims) fdtd_rom_destroy(s);
  delete bt;
}

}  // extern "C"
