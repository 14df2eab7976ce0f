// Batched runs (fdtd_rom_batch_*): B independent problems, each laid out by
// the single-problem path in its own slice of one device workspace, advanced
// together by one launch per step (batch_step_kernel) whose workgroups walk
// a table of (instance, role, index).  Table order: every instance's coupling
// blocks first (the longest workgroups start first), then each instance's
// stencil tiles from an index that is a multiple of 8 (so the XCD-aware tile
// remap of the single-problem kernel holds per instance), then one probe
// block per instance.  run() replays captured graphs of `graph_batch` steps.
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
};

int plan_batch(const fdtd_problem* probs, int B, BatchPlan& P) {
  if (!probs || B < 1) return fail(FDTD_EINVAL, "need at least one instance");
  const int dt = probs[0].grid.dtype;
  size_t cap = 8;
  P.inst_off.assign(B, 0);
  P.inst_bytes.assign(B, 0);
  std::vector<size_t> sizes(B);
  for (int b = 0; b < B; ++b) {
    if (probs[b].grid.dtype != dt) return fail(FDTD_EINVAL, "instance %d: every instance must share one dtype", b);
    Layout L;
    const int rc = plan_problem(&probs[b], L);
    if (rc != FDTD_OK) return fail(rc, "instance %d: %s", b, fdtd_rom_last_error());
    sizes[b] = L.total;
    cap += (size_t)std::max(L.nrowblocks, L.nblocks_mixed) + (size_t)tiles_for(probs[b], 4) + 7 + 1;
  }
  const size_t desc_bytes = (size_t)B * (dt == FDTD_F32 ? sizeof(StepParams<float>) : sizeof(StepParams<double>));
  size_t o = 0;
  P.off_ctrl = o;
  o = align_up(o + kCtrlInts * sizeof(int), 256);
  P.off_desc = o;
  o = align_up(o + desc_bytes, 256);
  P.off_table = o;
  P.table_cap = cap;
  o = align_up(o + cap * sizeof(BatchRef), 256);
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
  for (int b = 0; b < bt->B; ++b)
    for (int k = 0; k < nrow(b); ++k) t.push_back(BatchRef{b, 0, k, 0});
  for (int b = 0; b < bt->B; ++b) {
    pad8();
    for (int k = 0; k < ntile(b); ++k) t.push_back(BatchRef{b, 1, k, 0});
  }
  for (int b = 0; b < bt->B; ++b) t.push_back(BatchRef{b, 2, 0, 0});
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
  build_table(bt);
  if (bt->table.size() > bt->table_cap) return fail(FDTD_EINVAL, "internal: batch table overflow");
  std::vector<StepParams<T>> d(bt->B);
  for (int b = 0; b < bt->B; ++b) d[b] = step_params<T>(bt->sims[b]);
  if (hipMemcpyAsync(bt->ws + bt->off_desc, d.data(), d.size() * sizeof(StepParams<T>), hipMemcpyHostToDevice,
                     bt->stream) != hipSuccess ||
      hipMemcpyAsync(bt->ws + bt->off_table, bt->table.data(), bt->table.size() * sizeof(BatchRef),
                     hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
      hipStreamSynchronize(bt->stream) != hipSuccess)
    return fail(FDTD_EDEVICE, "batch descriptor upload failed");
  bt->dirty = false;
  return FDTD_OK;
}

template <typename T>
int enqueue_batch(fdtd_rom_batch* bt, int nsteps, hipStream_t st) {
  const StepParams<T>* d = (const StepParams<T>*)(bt->ws + bt->off_desc);
  const BatchRef* tab = (const BatchRef*)(bt->ws + bt->off_table);
  int* ctrl = (int*)(bt->ws + bt->off_ctrl);
  for (int k = 0; k < nsteps; ++k)
    if (launch_batch_step<T>(d, tab, (int)bt->table.size(), ctrl, k, bt->smem, bt->layers, bt->midx, st) !=
        hipSuccess)
      return fail(FDTD_EDEVICE, "batch step launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (launch_batch_probe_flush<T>(d, bt->B, ctrl, nsteps, st) != hipSuccess || launch_tick(ctrl, nsteps, st) != hipSuccess)
    return fail(FDTD_EDEVICE, "batch probe/tick launch failed");
  return FDTD_OK;
}

template <typename T>
int capture_batch(fdtd_rom_batch* bt) {
  drop_batch_graph(bt);
  if (!bt->cap_stream && hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamCreateWithFlags failed");
  if (hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail(FDTD_EDEVICE, "hipStreamBeginCapture failed");
  const int rc = enqueue_batch<T>(bt, bt->graph_batch, bt->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(bt->cap_stream, &g);
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
  bt->graph_steps = bt->graph_batch;
  return FDTD_OK;
}

template <typename T>
int run_batch(fdtd_rom_batch* bt, int nsteps) {
  if (bt->dirty) {
    drop_batch_graph(bt);
    const int rc = upload<T>(bt);
    if (rc != FDTD_OK) return rc;
  }
  int done = 0;
  if (bt->graph_batch > 0 && nsteps >= bt->graph_batch) {
    if (!bt->graph || bt->graph_steps != bt->graph_batch) {
      const int rc = capture_batch<T>(bt);
      if (rc != FDTD_OK) return rc;
    }
    while (nsteps - done >= bt->graph_batch) {
      if (hipGraphLaunch(bt->graph, bt->stream) != hipSuccess)
        return fail(FDTD_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(hipGetLastError()));
      done += bt->graph_batch;
    }
  }
  if (nsteps > done) {
    const int rc = enqueue_batch<T>(bt, nsteps - done, bt->stream);
    if (rc != FDTD_OK) return rc;
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
    for (int b = 0; b < B && rc == FDTD_OK; ++b) {
      fdtd_rom_sim* s = nullptr;
      rc = fdtd_rom_create(&probs[b], bt->ws + P.inst_off[b], P.inst_bytes[b], hip_stream, &s);
      if (rc != FDTD_OK) {
        rc = fail(rc, "instance %d: %s", b, fdtd_rom_last_error());
        break;
      }
      // a batch advances every instance by one launch per step
      s->tb = false;
      set_tiling(s, default_tiling(s->nx, s->ny, (int)s->L.tsize));
      bt->sims.push_back(s);
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
