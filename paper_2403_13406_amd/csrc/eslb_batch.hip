// Batched ensembles: many independent problems of one (lattice, system) kind and
// uneven grid sizes advanced together, one stage kernel per pass over all of them.
//
// Every instance runs the same composed-step schedule (eq. splittingToUse), so
// the ensemble advances in lockstep, pass by pass.  The grid of every instance is
// cut into tiles of one block; a device table maps tile -> instance.  Instances
// are sorted by their step counts, longest first, so at lockstep step s the active
// instances form a prefix and their tiles a prefix of the table.  The stage
// kernel covers the active tiles, either with a persistent grid of blocks that
// strides over them or with one block per tile of the whole table (the launch
// configuration, chosen by the autotuner); the active-tile count and the step
// counter live in device memory and are advanced by a small kernel at the end
// of each step, so one captured hipGraph of k steps replays until the longest
// instance is done, with no host work in between.
//
// Offsets: transport shifts every population by the same number of cells, so an
// instance needs one offset o (cells travelled); at pass p of lockstep step s,
// o = o_start + s * net + cum[p], kept modulo each instance's grid.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  int nx, ny;
  int ox0, oy0;    // offset of every population when the run starts, mod nx and mod ny
  int netx, nety;  // offset gained per composed step, mod nx and mod ny
  Phys P;
};

constexpr int kMaxPass = 64;  // passes per composed step the control block has queues for
struct BatchCtl {
  long long step;     // lockstep step counter
  int active_tiles;   // tiles of instances that still have steps to do
  int active;         // number of such instances
  unsigned next[kMaxPass];  // per pass: the next tile for the persistent grid (zeroed every step)
};

// Offsets are kept modulo the grid: omod[i] = (o mod nx, o mod ny) of instance i at
// the start of the current lockstep step (advanced by k_batch_advance), and
// cmod[i * npass + p] = (c_p mod nx, c_p mod ny), c_p the cells moved by this
// step's transports up to pass p.  A population's storage shift at pass p is then
// one addition and one conditional subtraction (no 64-bit division per tile).
struct TileRef {
  int inst, tx, ty, pad;
};

// Storage byte offset of population k of cell (x, y) for offsets m = o mod (nx, ny):
// logical f_k(x) sits at x - sign_k o along its axis.  A state is below 4 GiB
// (checked at creation), so every access is the instance's base pointer (scalar)
// plus a 32-bit byte offset.
template <int D>
__device__ __forceinline__ unsigned boffset(int k, int x, int y, int nx, int ny, int mx, int my) {
  int xs = x, ys = y;
  if (Lat<D>::axis(k) == 0) {
    xs += (Lat<D>::sign(k) > 0) ? (mx == 0 ? 0 : nx - mx) : mx;
    if (xs >= nx) xs -= nx;
  } else {
    ys += (Lat<D>::sign(k) > 0) ? (my == 0 ? 0 : ny - my) : my;
    if (ys >= ny) ys -= ny;
  }
  return ((unsigned)ys * (unsigned)nx + (unsigned)xs) * 8u;
}

// A state pointer read from the instance table is a generic pointer to the
// compiler (flat loads and stores, 64-bit per-lane addresses); the states live in
// global memory, so the accesses go through a global-address-space pointer: the
// plane's base is uniform (scalar registers) and each access is that base plus a
// 32-bit per-lane byte offset.
using gchar = __attribute__((address_space(1))) char;
using gdouble = __attribute__((address_space(1))) double;
__device__ __forceinline__ gdouble& bat(const gchar* plane, unsigned byte_off) {
  return *reinterpret_cast<gdouble*>(const_cast<gchar*>(plane) + byte_off);
}

// One relaxation pass (pass p of the step) over every active tile.  queue = 0:
// one block per tile of the whole table (blocks past the active prefix return at
// once).  queue = 1: a persistent grid whose blocks take tiles from the pass's
// counter (ctl->next[p]) until the active tiles are exhausted, so that blocks
// that drew cheap tiles (fast root searches) go on to take more.
template <class S, int D, int BX, int BY>
__global__ __launch_bounds__(BX* BY, S::kBatchBlocks) void k_batch_stage(const BatchInst* __restrict__ inst,
                                                          const TileRef* __restrict__ tiles, BatchCtl* ctl,
                                                          const int2* __restrict__ omod, const int2* __restrict__ cmod,
                                                          int npass, int p, int mode, int omega_one, int queue,
                                                          DevStats* st) {
  constexpr int Q = S::Q, M = S::M;
  __shared__ int next_tile;
  const int ntiles = ctl->active_tiles;
  int tile = (int)blockIdx.x;
  if (queue) {
    if (threadIdx.x == 0) next_tile = (int)atomicAdd(&ctl->next[p], 1u);
    __syncthreads();
    tile = next_tile;
  }
  for (;;) {
    if (tile >= ntiles) break;
    // the next tile is taken now, so that the atomic's round trip overlaps this tile's work
    int pre = 0;
    if (queue && threadIdx.x == 0) pre = (int)atomicAdd(&ctl->next[p], 1u);
    const TileRef tr = tiles[tile];
    const int i = tr.inst;
    const BatchInst& b = inst[i];
    const int x = tr.tx * BX + (int)(threadIdx.x % BX);
    const int y = tr.ty * BY + (int)(threadIdx.x / BX);
    if (x < b.nx && y < b.ny) {
      const int2 om = omod[i], cm = cmod[i * npass + p];
      int mx = om.x + cm.x, my = om.y + cm.y;
      if (mx >= b.nx) mx -= b.nx;
      if (my >= b.ny) my -= b.ny;
      const size_t pb = (size_t)b.nx * (size_t)b.ny * 8u;  // plane bytes
      const gchar* base = (const gchar*)b.f;
      unsigned off[Q];
      double f[Q][M];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        off[k] = boffset<D>(k, x, y, b.nx, b.ny, mx, my);
#pragma unroll
        for (int m = 0; m < M; ++m) f[k][m] = bat(base + (k * M + m) * pb, off[k]);
      }
      unsigned flags = 0;
      Phys P = b.P;
      if (omega_one) P.omega = 1.0;
      relax_node<S>(f, mode, P, flags);
      // offsets as 32-bit values of this block (see k_stage)
#pragma unroll
      for (int k = 0; k < Q; ++k) asm volatile("" : "+v"(off[k]));
      bool fin = true;
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          fin &= isfinite(f[k][m]);
          bat(base + (k * M + m) * pb, off[k]) = f[k][m];
        }
      if (!fin) flags |= FLAG_NAN;
      if (flags) {
        atomicOr(&st->flags, flags);
        if (flags & FLAG_FALLBACK) atomicAdd(&st->n_fallback, 1ull);
      }
    }
    if (!queue) break;
    __syncthreads();  // every thread has read next_tile before it is overwritten
    if (threadIdx.x == 0) next_tile = pre;
    __syncthreads();
    tile = next_tile;
  }
}

// End of a lockstep step: every instance's offsets move by one step (mod the
// grid); thread 0 advances the counter and shrinks the active prefix.
__global__ void k_batch_advance(BatchCtl* ctl, const long long* __restrict__ steps_sorted,
                                const int* __restrict__ tiles_prefix, const BatchInst* __restrict__ inst,
                                int2* __restrict__ omod, int n, int npass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const BatchInst& b = inst[i];
    int2 o = omod[i];
    o.x += b.netx;
    if (o.x >= b.nx) o.x -= b.nx;
    o.y += b.nety;
    if (o.y >= b.ny) o.y -= b.ny;
    omod[i] = o;
  }
  if (i == 0) {
    const long long s = ctl->step + 1;
    int a = ctl->active;
    while (a > 0 && steps_sorted[a - 1] <= s) --a;
    ctl->step = s;
    ctl->active = a;
    ctl->active_tiles = tiles_prefix[a];
    for (int q = 0; q < npass; ++q) ctl->next[q] = 0u;
  }
}

__global__ void k_batch_reset(BatchCtl* ctl, int active, int tiles, const BatchInst* __restrict__ inst,
                              int2* __restrict__ omod, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) omod[i] = make_int2(inst[i].ox0, inst[i].oy0);
  if (i == 0) {
    ctl->step = 0;
    ctl->active = active;
    ctl->active_tiles = tiles;
    for (int q = 0; q < kMaxPass; ++q) ctl->next[q] = 0u;
  }
}

// blocks_per_cu = 0: one block per tile of the whole table (the blocks past the
// active prefix return at once), so the hardware dispatcher balances the tiles
// whose root searches take longer; otherwise a persistent grid of that many
// blocks per CU that takes tiles from a per-pass queue.
struct Config {
  int bx, by, blocks_per_cu;
};

const Config kConfigs[] = {{64, 4, 8}, {64, 4, 4}, {64, 4, 16}, {128, 2, 8}, {256, 1, 8}, {32, 8, 8},
                           {64, 2, 8}, {64, 4, 0}, {64, 2, 0}, {128, 1, 0}, {128, 1, 8}};

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
void launch_cfg(const Config& c, int grid, hipStream_t st, const BatchInst* inst, const TileRef* tiles,
                BatchCtl* ctl, const int2* omod, const int2* cmod, int npass, int p, int mode, int om1,
                DevStats* ds) {
  const int queue = c.blocks_per_cu > 0 ? 1 : 0;
#define L(BX, BY)                                                                                                  \
  hipLaunchKernelGGL((k_batch_stage<S, D, BX, BY>), dim3(grid), dim3(BX * BY), 0, st, inst, tiles, ctl, omod, cmod, \
                     npass, p, mode, om1, queue, ds)
  if (c.bx == 64 && c.by == 4) L(64, 4);
  else if (c.bx == 128 && c.by == 2) L(128, 2);
  else if (c.bx == 256 && c.by == 1) L(256, 1);
  else if (c.bx == 32 && c.by == 8) L(32, 8);
  else if (c.bx == 64 && c.by == 2) L(64, 2);
  else if (c.bx == 128 && c.by == 1) L(128, 1);
#undef L
}

void launch_kind(int kind, const Config& c, int grid, hipStream_t st, const BatchInst* inst, const TileRef* tiles,
                 BatchCtl* ctl, const int2* omod, const int2* cmod, int npass, int p, int mode, int om1,
                 DevStats* ds) {
#define CALL(S, D) launch_cfg<S, D>(c, grid, st, inst, tiles, ctl, omod, cmod, npass, p, mode, om1, ds)
  ESLB_DISPATCH_KIND(kind, CALL)
#undef CALL
}

// Device tables for one run over `order` (instance ids sorted by steps, longest first).
struct RunTables {
  BatchInst* inst = nullptr;
  TileRef* tiles = nullptr;
  int* tiles_prefix = nullptr;
  long long* steps_sorted = nullptr;
  int2* omod = nullptr;
  int2* cmod = nullptr;
  BatchCtl* ctl = nullptr;
  int ntiles = 0, nact = 0;
  long long max_steps = 0;
  void release() {
    (void)hipFree(inst);
    (void)hipFree(tiles);
    (void)hipFree(tiles_prefix);
    (void)hipFree(steps_sorted);
    (void)hipFree(omod);
    (void)hipFree(cmod);
    (void)hipFree(ctl);
    *this = RunTables();
  }
};

long long pmod_ll(long long a, long long n) {
  const long long r = a % n;
  return r < 0 ? r + n : r;
}

int build_tables(eslb_batch* b, const Config& cfg, double* const* f, const std::vector<int>& order,
                 const std::vector<long long>& steps, RunTables& T) {
  const int n = (int)order.size();
  const eslb_ctx* c = b->proto;
  const int npass = (int)c->passes.size();
  if (npass > kMaxPass) return berr(b, ESLB_ERR_INVALID_ARG, "batch: schedule has more passes per step than supported");
  const long long net = net_shift(c);
  std::vector<BatchInst> hi(n);
  std::vector<int> first(n + 1, 0), prefix(n + 1, 0);
  std::vector<long long> ss(n);
  std::vector<int2> cm((size_t)n * npass);
  for (int r = 0; r < n; ++r) {
    const int i = order[r];
    const eslb_problem& p = b->probs[i];
    BatchInst& d = hi[r];
    d.f = f[i];
    d.nx = p.nx;
    d.ny = p.ny;
    d.ox0 = (int)pmod_ll(b->offs[i], p.nx);
    d.oy0 = (int)pmod_ll(b->offs[i], p.ny);
    d.netx = (int)pmod_ll(net, p.nx);
    d.nety = (int)pmod_ll(net, p.ny);
    d.P = make_phys(p, b->q);
    long long cum = 0;
    for (int q = 0; q < npass; ++q) {
      cum += c->passes[q].shift;
      cm[(size_t)r * npass + q] = make_int2((int)pmod_ll(cum, p.nx), (int)pmod_ll(cum, p.ny));
    }
    const int tx = (p.nx + cfg.bx - 1) / cfg.bx;
    const int tiles = tx * ((p.ny + cfg.by - 1) / cfg.by);
    first[r + 1] = first[r] + tiles;
    prefix[r + 1] = first[r + 1];
    ss[r] = steps[i];
  }
  T.ntiles = first[n];
  T.nact = n;
  T.max_steps = n ? ss[0] : 0;
  std::vector<TileRef> tt((size_t)std::max(T.ntiles, 1));
  for (int r = 0; r < n; ++r) {
    const int tx = (hi[r].nx + cfg.bx - 1) / cfg.bx;
    for (int t = first[r]; t < first[r + 1]; ++t) {
      const int lt = t - first[r];
      tt[t] = TileRef{r, lt % tx, lt / tx, 0};
    }
  }
  hipError_t e = hipSuccess;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(dst, std::max<size_t>(bytes, 16));
    if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  up((void**)&T.inst, hi.data(), sizeof(BatchInst) * n);
  up((void**)&T.tiles, tt.data(), sizeof(TileRef) * tt.size());
  up((void**)&T.tiles_prefix, prefix.data(), sizeof(int) * prefix.size());
  up((void**)&T.steps_sorted, ss.data(), sizeof(long long) * n);
  up((void**)&T.cmod, cm.data(), sizeof(int2) * cm.size());
  if (e == hipSuccess) e = hipMalloc(&T.omod, sizeof(int2) * std::max(n, 1));
  if (e == hipSuccess) e = hipMalloc(&T.ctl, sizeof(BatchCtl));
  if (e != hipSuccess) {
    T.release();
    return bhip(b, e, "batch tables");
  }
  return ESLB_OK;
}

int capture_steps(eslb_batch* b, const Config& cfg, const RunTables& T, int k, hipGraphExec_t* exec) {
  eslb_ctx* c = b->proto;
  const int npass = (int)c->passes.size();
  const int grid = std::max(1, cfg.blocks_per_cu > 0 ? std::min(T.ntiles, b->cus * cfg.blocks_per_cu) : T.ntiles);
  hipGraph_t g = nullptr;
  int rc = bhip(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc != ESLB_OK) return rc;
  for (int s = 0; s < k; ++s) {
    for (int p = 0; p < npass; ++p) {
      const Pass& ps = c->passes[p];
      const int mode = (ps.op == PASS_PROJECT) ? 0 : c->pb.relax;
      launch_kind(b->kind, cfg, grid, b->cap, T.inst, T.tiles, T.ctl, T.omod, T.cmod, npass, p, mode,
                  ps.op == PASS_PROJECT ? 1 : 0, c->st);
    }
    hipLaunchKernelGGL(k_batch_advance, dim3((T.nact + 255) / 256), dim3(256), 0, b->cap, T.ctl, T.steps_sorted,
                       T.tiles_prefix, T.inst, T.omod, T.nact, npass);
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
    hipLaunchKernelGGL(k_batch_reset, dim3((T.nact + 255) / 256), dim3(256), 0, b->cap, T.ctl, T.nact, T.ntiles,
                       T.inst, T.omod, T.nact);
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
    if ((long long)q * M * p.nx * p.ny * (long long)sizeof(double) >= (1ll << 32)) {
      eslb_batch_destroy(b);
      return berr(nullptr, ESLB_ERR_INVALID_ARG, "problem " + std::to_string(i) + ": batch instance states must be below 4 GiB");
    }
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
      if (blocks_per_cu < 0 || steps_per_graph < 1) break;
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

int eslb_batch_autotune(eslb_batch* b, double* const* f, int32_t replays, double* best_ms) {
  if (!b || !f || replays < 1) return berr(b, ESLB_ERR_INVALID_ARG, "bad argument to eslb_batch_autotune");
  replays = std::max(replays, 3);
  // Tuning set: a systematic sample of at most kTuneInstances instances taken
  // along the ensemble sorted by grid size, so the tile mix is in proportion to
  // the ensemble's size distribution.  They run on scratch copies (the caller's
  // states and offsets are untouched).
  constexpr int kTuneInstances = 64;
  const int n = (int)b->probs.size();
  std::vector<int> by_size;
  for (int i = 0; i < n; ++i)
    if (f[i]) by_size.push_back(i);
  if (by_size.empty()) return berr(b, ESLB_ERR_INVALID_ARG, "no state to tune on");
  std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int c) {
    return (long long)b->probs[a].nx * b->probs[a].ny < (long long)b->probs[c].nx * b->probs[c].ny;
  });
  const int nsamp = std::min((int)by_size.size(), kTuneInstances);
  std::vector<int> reps;
  for (int j = 0; j < nsamp; ++j) reps.push_back(by_size[(size_t)j * by_size.size() / nsamp]);
  std::vector<double*> scratch(n, nullptr);
  int rc = ESLB_OK;
  for (int i : reps) {
    const size_t bytes = (size_t)b->q * b->M * b->probs[i].nx * (size_t)b->probs[i].ny * sizeof(double);
    rc = bhip(b, hipMalloc(&scratch[i], bytes), "autotune scratch");
    if (rc == ESLB_OK) rc = bhip(b, hipMemcpyAsync(scratch[i], f[i], bytes, hipMemcpyDeviceToDevice, b->stream), "copy");
    if (rc != ESLB_OK) break;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (rc == ESLB_OK) rc = bhip(b, hipEventCreate(&e0), "event");
  if (rc == ESLB_OK) rc = bhip(b, hipEventCreate(&e1), "event");
  if (rc == ESLB_OK) rc = bhip(b, hipStreamSynchronize(b->stream), "sync");
  // every sampled instance stays active through the warm-up and timed replays
  std::vector<long long> steps(n, 0);
  for (int i : reps) steps[i] = replays + 2;
  const std::vector<int> order = sorted_order(steps, reps);
  double best = 1e300;
  Config best_cfg = b->cfg;
  for (const Config& c : kConfigs) {
    if (rc != ESLB_OK) break;
    // tables and a one-step graph once per configuration; only graph replays are timed
    RunTables T;
    rc = build_tables(b, c, scratch.data(), order, steps, T);
    if (rc != ESLB_OK) break;
    hipGraphExec_t exec = nullptr;
    rc = capture_steps(b, c, T, 1, &exec);
    if (rc == ESLB_OK) {
      hipLaunchKernelGGL(k_batch_reset, dim3((T.nact + 255) / 256), dim3(256), 0, b->cap, T.ctl, T.nact, T.ntiles,
                         T.inst, T.omod, T.nact);
      rc = bhip(b, hipGetLastError(), "reset launch");
    }
    if (rc == ESLB_OK) rc = bhip(b, hipGraphLaunch(exec, b->cap), "graph launch");  // warm-up
    double ms = 1e300;
    for (int r = 0; r < replays && rc == ESLB_OK; ++r) {
      rc = bhip(b, hipEventRecord(e0, b->cap), "event record");
      if (rc == ESLB_OK) rc = bhip(b, hipGraphLaunch(exec, b->cap), "graph launch");
      if (rc == ESLB_OK) rc = bhip(b, hipEventRecord(e1, b->cap), "event record");
      if (rc == ESLB_OK) rc = bhip(b, hipEventSynchronize(e1), "event sync");
      float t = 0.f;
      if (rc == ESLB_OK) rc = bhip(b, hipEventElapsedTime(&t, e0, e1), "event time");
      if (rc == ESLB_OK) ms = std::min(ms, (double)t);
    }
    if (rc == ESLB_OK) rc = bhip(b, hipStreamSynchronize(b->cap), "sync");
    if (exec) (void)hipGraphExecDestroy(exec);
    T.release();
    if (rc == ESLB_OK && ms < best) {
      best = ms;
      best_cfg = c;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int i : reps) (void)hipFree(scratch[i]);
  if (rc != ESLB_OK) return rc;
  b->cfg = best_cfg;
  if (best_ms) *best_ms = best;
  return ESLB_OK;
}

const char* eslb_batch_last_error(const eslb_batch* b) { return b ? b->err.c_str() : eslb_last_error(nullptr); }

}  // extern "C"
