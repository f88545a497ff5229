// Batched ensembles: many independent problems of one (lattice, system) kind and
// uneven grid sizes advanced together by one persistent stage kernel.
//
// Every instance runs the same composed-step schedule (eq. splittingToUse), so
// the ensemble advances in lockstep, pass by pass.  The grid of every instance is
// cut into tiles of one block; a device table maps tile -> instance.  Instances
// are sorted by their step counts, longest first, so at lockstep step s the active
// instances form a prefix and their tiles a prefix of the table.  A persistent
// grid of blocks strides over the active tiles; the active-tile count and the step
// counter live in device memory and are advanced by a one-thread kernel at the end
// of each step, so one captured hipGraph of k steps replays until the longest
// instance is done, with no host work in between.
//
// Offsets: transport shifts every population by the same number of cells, so an
// instance needs one offset o (cells travelled); at pass p of lockstep step s,
// o = o_start + s * net + cum[p].  Storage shifts follow per instance (mod nx, ny).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "eslb.h"
#include "eslb_internal.hpp"
#include "eslb_systems.hpp"

using namespace eslb;

namespace {

struct BatchInst {
  double* f;
  long long plane;
  int nx, ny;
  int tiles_x;
  int pad;
  long long o_start;  // offset of every population when the run starts
  Phys P;
};

struct BatchCtl {
  long long step;     // lockstep step counter
  int active_tiles;   // tiles of instances that still have steps to do
  int active;         // number of such instances
};

template <int D>
__device__ __forceinline__ long long bstorage(const BatchInst& b, int k, int x, int y, int shx, int shy) {
  const int sh = (Lat<D>::axis(k) == 0) ? (Lat<D>::sign(k) > 0 ? shx : (shx == 0 ? 0 : b.nx - shx))
                                        : (Lat<D>::sign(k) > 0 ? shy : (shy == 0 ? 0 : b.ny - shy));
  if (Lat<D>::axis(k) == 0) {
    int xs = x + sh;
    if (xs >= b.nx) xs -= b.nx;
    return (long long)y * b.nx + xs;
  }
  int ys = y + sh;
  if (ys >= b.ny) ys -= b.ny;
  return (long long)ys * b.nx + x;
}

// One relaxation pass over every active tile.  cum: cells moved by the transports
// of this step up to and including the one before this pass.
template <class S, int D, int BX, int BY>
__global__ __launch_bounds__(BX* BY, 2) void k_batch_stage(const BatchInst* __restrict__ inst,
                                                          const int* __restrict__ tile_inst,
                                                          const int* __restrict__ tile_first, const BatchCtl* ctl,
                                                          long long net, long long cum, int mode, int omega_one,
                                                          DevStats* st) {
  constexpr int Q = S::Q, M = S::M;
  const int ntiles = ctl->active_tiles;
  const long long step = ctl->step;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i = tile_inst[tile];
    const BatchInst& b = inst[i];
    const int lt = tile - tile_first[i];
    const int tx = lt % b.tiles_x, ty = lt / b.tiles_x;
    const int x = tx * BX + (int)(threadIdx.x % BX);
    const int y = ty * BY + (int)(threadIdx.x / BX);
    if (x >= b.nx || y >= b.ny) continue;
    const long long o = b.o_start + step * net + cum;
    // storage shift of a + velocity along x is (-o) mod nx; of a - velocity, (+o) mod nx
    long long mx = o % b.nx;
    if (mx < 0) mx += b.nx;
    long long my = o % b.ny;
    if (my < 0) my += b.ny;
    const int shx = (int)((b.nx - mx) % b.nx), shy = (int)((b.ny - my) % b.ny);
    long long id[Q];
    double f[Q][M];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      id[k] = bstorage<D>(b, k, x, y, shx, shy);
#pragma unroll
      for (int m = 0; m < M; ++m) f[k][m] = b.f[(long long)(k * M + m) * b.plane + id[k]];
    }
    unsigned flags = 0;
    Phys P = b.P;
    if (omega_one) P.omega = 1.0;
    relax_node<S>(f, mode, P, flags);
    bool fin = true;
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < M; ++m) {
        fin &= isfinite(f[k][m]);
        b.f[(long long)(k * M + m) * b.plane + id[k]] = f[k][m];
      }
    if (!fin) flags |= FLAG_NAN;
    if (flags) {
      atomicOr(&st->flags, flags);
      if (flags & FLAG_FALLBACK) atomicAdd(&st->n_fallback, 1ull);
    }
  }
}

// End of a lockstep step: advance the counter and shrink the active prefix.
__global__ void k_batch_advance(BatchCtl* ctl, const long long* __restrict__ steps_sorted,
                                const int* __restrict__ tiles_prefix) {
  const long long s = ctl->step + 1;
  int a = ctl->active;
  while (a > 0 && steps_sorted[a - 1] <= s) --a;
  ctl->step = s;
  ctl->active = a;
  ctl->active_tiles = tiles_prefix[a];
}

__global__ void k_batch_reset(BatchCtl* ctl, int active, int tiles) {
  ctl->step = 0;
  ctl->active = active;
  ctl->active_tiles = tiles;
}

struct Config {
  int bx, by, blocks_per_cu;
};

const Config kConfigs[] = {{64, 4, 8}, {64, 4, 4}, {64, 4, 16}, {128, 2, 8}, {256, 1, 8}, {32, 8, 8}, {64, 2, 8}};

}  // namespace

struct eslb_batch {
  std::vector<eslb_problem> probs;
  std::vector<long long> offs;  // per-instance offset (every population)
  int kind = 0, d = 2, q = 4, M = 1;
  hipStream_t stream = nullptr;  // caller's stream
  hipStream_t cap = nullptr;     // library stream used for capture
  eslb_ctx* proto = nullptr;     // context of instance 0 (schedule, status block)
  int cus = 256;
  Config cfg{64, 4, 8};
  int steps_per_graph = 8;
  std::string err;
};

namespace {

int berr(eslb_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  eslb_set_global_error(m);
  return code;
}

int bhip(eslb_batch* b, hipError_t e, const char* what) {
  if (e == hipSuccess) return ESLB_OK;
  return berr(b, ESLB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class S, int D>
void launch_cfg(const Config& c, int grid, hipStream_t st, const BatchInst* inst, const int* ti, const int* tf,
                const BatchCtl* ctl, long long net, long long cum, int mode, int om1, DevStats* ds) {
#define L(BX, BY)                                                                                               \
  hipLaunchKernelGGL((k_batch_stage<S, D, BX, BY>), dim3(grid), dim3(BX * BY), 0, st, inst, ti, tf, ctl, net, cum, \
                     mode, om1, ds)
  if (c.bx == 64 && c.by == 4) L(64, 4);
  else if (c.bx == 128 && c.by == 2) L(128, 2);
  else if (c.bx == 256 && c.by == 1) L(256, 1);
  else if (c.bx == 32 && c.by == 8) L(32, 8);
  else if (c.bx == 64 && c.by == 2) L(64, 2);
#undef L
}

void launch_kind(int kind, const Config& c, int grid, hipStream_t st, const BatchInst* inst, const int* ti,
                 const int* tf, const BatchCtl* ctl, long long net, long long cum, int mode, int om1, DevStats* ds) {
#define CALL(S, D) launch_cfg<S, D>(c, grid, st, inst, ti, tf, ctl, net, cum, mode, om1, ds)
  ESLB_DISPATCH_KIND(kind, CALL)
#undef CALL
}

// Device tables for one run over `order` (instance ids sorted by steps, longest first).
struct RunTables {
  BatchInst* inst = nullptr;
  int* tile_inst = nullptr;
  int* tile_first = nullptr;
  int* tiles_prefix = nullptr;
  long long* steps_sorted = nullptr;
  BatchCtl* ctl = nullptr;
  int ntiles = 0, nact = 0;
  long long max_steps = 0;
  void release() {
    (void)hipFree(inst);
    (void)hipFree(tile_inst);
    (void)hipFree(tile_first);
    (void)hipFree(tiles_prefix);
    (void)hipFree(steps_sorted);
    (void)hipFree(ctl);
    *this = RunTables();
  }
};

int build_tables(eslb_batch* b, const Config& cfg, double* const* f, const std::vector<int>& order,
                 const std::vector<long long>& steps, RunTables& T) {
  const int n = (int)order.size();
  std::vector<BatchInst> hi(n);
  std::vector<int> first(n + 1, 0), prefix(n + 1, 0);
  std::vector<long long> ss(n);
  for (int r = 0; r < n; ++r) {
    const int i = order[r];
    const eslb_problem& p = b->probs[i];
    BatchInst& d = hi[r];
    d.f = f[i];
    d.nx = p.nx;
    d.ny = p.ny;
    d.plane = (long long)p.nx * p.ny;
    d.tiles_x = (p.nx + cfg.bx - 1) / cfg.bx;
    d.pad = 0;
    d.o_start = b->offs[i];
    d.P = make_phys(p, b->q);
    const int tiles = d.tiles_x * ((p.ny + cfg.by - 1) / cfg.by);
    first[r + 1] = first[r] + tiles;
    prefix[r + 1] = first[r + 1];
    ss[r] = steps[i];
  }
  T.ntiles = first[n];
  T.nact = n;
  T.max_steps = n ? ss[0] : 0;
  std::vector<int> ti((size_t)std::max(T.ntiles, 1));
  for (int r = 0; r < n; ++r)
    for (int t = first[r]; t < first[r + 1]; ++t) ti[t] = r;
  hipError_t e = hipSuccess;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(dst, std::max<size_t>(bytes, 16));
    if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  up((void**)&T.inst, hi.data(), sizeof(BatchInst) * n);
  up((void**)&T.tile_inst, ti.data(), sizeof(int) * ti.size());
  up((void**)&T.tile_first, first.data(), sizeof(int) * first.size());
  up((void**)&T.tiles_prefix, prefix.data(), sizeof(int) * prefix.size());
  up((void**)&T.steps_sorted, ss.data(), sizeof(long long) * n);
  if (e == hipSuccess) e = hipMalloc(&T.ctl, sizeof(BatchCtl));
  if (e != hipSuccess) {
    T.release();
    return bhip(b, e, "batch tables");
  }
  return ESLB_OK;
}

int capture_steps(eslb_batch* b, const Config& cfg, const RunTables& T, int k, hipGraphExec_t* exec) {
  eslb_ctx* c = b->proto;
  const long long net = net_shift(c);
  const int grid = std::max(1, std::min(T.ntiles, b->cus * cfg.blocks_per_cu));
  hipGraph_t g = nullptr;
  int rc = bhip(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc != ESLB_OK) return rc;
  for (int s = 0; s < k; ++s) {
    long long cum = 0;
    for (const Pass& p : c->passes) {
      cum += p.shift;
      const int mode = (p.op == PASS_PROJECT) ? 0 : c->pb.relax;
      launch_kind(b->kind, cfg, grid, b->cap, T.inst, T.tile_inst, T.tile_first, T.ctl, net, cum, mode,
                  p.op == PASS_PROJECT ? 1 : 0, c->st);
    }
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(1), 0, b->cap, T.ctl, T.steps_sorted, T.tiles_prefix);
  }
  rc = bhip(b, hipStreamEndCapture(b->cap, &g), "end capture");
  if (rc != ESLB_OK) return rc;
  rc = bhip(b, hipGraphInstantiate(exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  return rc;
}

// Advance instances `order` (sorted, longest first) by steps[i] in lockstep.
int run_sorted(eslb_batch* b, const Config& cfg, double* const* f, const std::vector<int>& order,
               const std::vector<long long>& steps) {
  if (order.empty()) return ESLB_OK;
  RunTables T;
  int rc = build_tables(b, cfg, f, order, steps, T);
  if (rc != ESLB_OK) return rc;
  const int k = (int)std::max<long long>(1, std::min<long long>(b->steps_per_graph, T.max_steps));
  hipGraphExec_t exec = nullptr;
  rc = capture_steps(b, cfg, T, k, &exec);
  hipEvent_t ev = nullptr;
  if (rc == ESLB_OK) rc = bhip(b, hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  // order after the caller's earlier work on its stream
  if (rc == ESLB_OK) rc = bhip(b, hipEventRecord(ev, b->stream), "event record");
  if (rc == ESLB_OK) rc = bhip(b, hipStreamWaitEvent(b->cap, ev, 0), "stream wait");
  if (rc == ESLB_OK) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, b->cap, T.ctl, T.nact, T.ntiles);
    rc = bhip(b, hipGetLastError(), "reset launch");
  }
  for (long long done = 0; rc == ESLB_OK && done < T.max_steps; done += k)
    rc = bhip(b, hipGraphLaunch(exec, b->cap), "graph launch");
  if (rc == ESLB_OK) rc = bhip(b, hipEventRecord(ev, b->cap), "event record");
  if (rc == ESLB_OK) rc = bhip(b, hipStreamWaitEvent(b->stream, ev, 0), "stream wait");
  // the tables must outlive the graph's execution
  if (rc == ESLB_OK) rc = bhip(b, hipStreamSynchronize(b->cap), "batch synchronize");
  if (exec) (void)hipGraphExecDestroy(exec);
  if (ev) (void)hipEventDestroy(ev);
  T.release();
  if (rc == ESLB_OK) {
    const long long net = net_shift(b->proto);
    for (int i : order) b->offs[i] += steps[i] * net;
  }
  return rc;
}

std::vector<int> sorted_order(const std::vector<long long>& steps, const std::vector<int>& subset) {
  std::vector<int> o;
  for (int i : subset)
    if (steps[i] > 0) o.push_back(i);
  std::stable_sort(o.begin(), o.end(), [&](int a, int c) { return steps[a] > steps[c]; });
  return o;
}

}  // namespace

extern "C" {

int eslb_batch_create(const eslb_problem* probs, int32_t n, void* stream, eslb_batch** out) {
  if (!out || !probs || n < 1) return berr(nullptr, ESLB_ERR_INVALID_ARG, "batch needs at least one problem");
  *out = nullptr;
  eslb_ctx* proto = nullptr;
  int rc = eslb_create(&probs[0], stream, &proto);
  if (rc != ESLB_OK) return rc;
  eslb_batch* b = new eslb_batch();
  b->proto = proto;
  b->kind = proto->kind;
  b->d = proto->d;
  b->q = proto->q;
  b->M = proto->M;
  b->stream = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    std::string why;
    int kind = 0, d = 0, q = 0, M = 0;
    rc = validate_problem(&probs[i], why, &kind, &d, &q, &M);
    if (rc != ESLB_OK) {
      eslb_batch_destroy(b);
      return berr(nullptr, rc, "problem " + std::to_string(i) + ": " + why);
    }
    const eslb_problem& p = probs[i];
    if (kind != b->kind || p.relax != probs[0].relax || p.scheme != probs[0].scheme || p.kappa != probs[0].kappa) {
      eslb_batch_destroy(b);
      return berr(nullptr, ESLB_ERR_INVALID_ARG,
                  "batch problems must share lattice, system, relax mode, scheme and kappa");
    }
    b->probs.push_back(p);
    b->offs.push_back(0);
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->cus = prop.multiProcessorCount;
  rc = bhip(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "stream create");
  if (rc != ESLB_OK) {
    eslb_batch_destroy(b);
    return rc;
  }
  *out = b;
  return ESLB_OK;
}

void eslb_batch_destroy(eslb_batch* b) {
  if (!b) return;
  if (b->cap) {
    (void)hipStreamSynchronize(b->cap);
    (void)hipStreamDestroy(b->cap);
  }
  if (b->proto) eslb_destroy(b->proto);
  delete b;
}

int eslb_batch_run(eslb_batch* b, double* const* f, const int64_t* nsteps) {
  if (!b || !f || !nsteps) return berr(b, ESLB_ERR_INVALID_ARG, "NULL argument");
  const int n = (int)b->probs.size();
  std::vector<long long> steps(n);
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) {
    if (nsteps[i] < 0) return berr(b, ESLB_ERR_INVALID_ARG, "negative step count");
    if (nsteps[i] > 0 && !f[i]) return berr(b, ESLB_ERR_INVALID_ARG, "NULL state");
    steps[i] = nsteps[i];
    all[i] = i;
  }
  return run_sorted(b, b->cfg, f, sorted_order(steps, all), steps);
}

int eslb_batch_get_offsets(const eslb_batch* b, int32_t i, int64_t* offsets) {
  if (!b || !offsets || i < 0 || i >= (int)b->probs.size()) return ESLB_ERR_INVALID_ARG;
  for (int k = 0; k < b->q; ++k) offsets[k] = b->offs[i];
  return ESLB_OK;
}

int eslb_batch_set_offsets(eslb_batch* b, int32_t i, const int64_t* offsets) {
  if (!b || !offsets || i < 0 || i >= (int)b->probs.size()) return ESLB_ERR_INVALID_ARG;
  for (int k = 1; k < b->q; ++k)
    if (offsets[k] != offsets[0]) return berr(b, ESLB_ERR_INVALID_ARG, "batch offsets must be equal across velocities");
  b->offs[i] = offsets[0];
  return ESLB_OK;
}

int eslb_batch_sync_status(eslb_batch* b) {
  if (!b) return ESLB_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(b->cap);
  return eslb_sync_status(b->proto);
}

int eslb_batch_set_config(eslb_batch* b, int32_t block_x, int32_t block_y, int32_t blocks_per_cu, int32_t steps_per_graph) {
  if (!b) return ESLB_ERR_INVALID_ARG;
  for (const Config& c : kConfigs) {
    if (c.bx == block_x && c.by == block_y) {
      if (blocks_per_cu < 1 || steps_per_graph < 1) break;
      b->cfg = Config{block_x, block_y, blocks_per_cu};
      b->steps_per_graph = steps_per_graph;
      return ESLB_OK;
    }
  }
  return berr(b, ESLB_ERR_INVALID_ARG, "unsupported batch configuration");
}

int eslb_batch_get_config(const eslb_batch* b, int32_t* cfg) {
  if (!b || !cfg) return ESLB_ERR_INVALID_ARG;
  cfg[0] = b->cfg.bx;
  cfg[1] = b->cfg.by;
  cfg[2] = b->cfg.blocks_per_cu;
  cfg[3] = b->steps_per_graph;
  return ESLB_OK;
}

int eslb_batch_autotune(eslb_batch* b, double* const* f, int32_t trial_steps, double* best_ms) {
  if (!b || !f || trial_steps < 1) return berr(b, ESLB_ERR_INVALID_ARG, "bad argument to eslb_batch_autotune");
  // One representative instance per distinct grid size, copied to scratch so the
  // caller's states are untouched; every candidate runs the same trial.
  const int n = (int)b->probs.size();
  std::vector<int> reps;
  for (int i = 0; i < n; ++i) {
    bool seen = false;
    for (int r : reps) seen |= (b->probs[r].nx == b->probs[i].nx && b->probs[r].ny == b->probs[i].ny);
    if (!seen && f[i]) reps.push_back(i);
  }
  if (reps.empty()) return berr(b, ESLB_ERR_INVALID_ARG, "no state to tune on");
  std::vector<double*> scratch(n, nullptr), orig(n, nullptr);
  int rc = ESLB_OK;
  for (int i : reps) {
    size_t bytes = (size_t)b->q * b->M * b->probs[i].nx * (size_t)b->probs[i].ny * sizeof(double);
    rc = bhip(b, hipMalloc(&orig[i], bytes), "autotune scratch");
    if (rc == ESLB_OK) rc = bhip(b, hipMalloc(&scratch[i], bytes), "autotune scratch");
    if (rc == ESLB_OK) rc = bhip(b, hipMemcpyAsync(orig[i], f[i], bytes, hipMemcpyDeviceToDevice, b->stream), "copy");
    if (rc != ESLB_OK) break;
  }
  std::vector<long long> keep_offs = b->offs;
  std::vector<long long> steps(n, 0);
  for (int i : reps) steps[i] = trial_steps;
  double best = 1e300;
  Config best_cfg = b->cfg;
  for (const Config& c : kConfigs) {
    if (rc != ESLB_OK) break;
    double ms = 0.0;
    for (int rep = 0; rep < 2 && rc == ESLB_OK; ++rep) {  // the first round warms up
      for (int i : reps) {
        size_t bytes = (size_t)b->q * b->M * b->probs[i].nx * (size_t)b->probs[i].ny * sizeof(double);
        rc = bhip(b, hipMemcpyAsync(scratch[i], orig[i], bytes, hipMemcpyDeviceToDevice, b->stream), "copy");
      }
      if (rc == ESLB_OK) rc = bhip(b, hipStreamSynchronize(b->stream), "sync");
      b->offs = keep_offs;
      const auto t0 = std::chrono::steady_clock::now();
      if (rc == ESLB_OK) rc = run_sorted(b, c, scratch.data(), sorted_order(steps, reps), steps);
      const auto t1 = std::chrono::steady_clock::now();
      ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (rc == ESLB_OK && ms < best) {
      best = ms;
      best_cfg = c;
    }
  }
  b->offs = keep_offs;
  for (int i : reps) {
    (void)hipFree(scratch[i]);
    (void)hipFree(orig[i]);
  }
  if (rc != ESLB_OK) return rc;
  b->cfg = best_cfg;
  if (best_ms) *best_ms = best;
  return ESLB_OK;
}

const char* eslb_batch_last_error(const eslb_batch* b) { return b ? b->err.c_str() : eslb_last_error(nullptr); }

}  // extern "C"
