// libeslb: C ABI and HIP kernels of the fourth-order entropy-stable lattice
// Boltzmann time loop (Bellotti, Helluy, Navoret, arXiv 2403.13406) for gfx950.
//
// Design (MI355X):
//  * SoA state, q*M planes of nx*ny binary64, x fastest.
//  * Transport (eq. transportPhase) is integer shifts of whole planes; it is
//    kept as per-velocity offsets and folded into the addressing of the next
//    relaxation pass, so a stage "shift then relax" is exactly one read and one
//    write of every population, in place.  Along x the shifted read of a row is
//    contiguous except at the periodic wrap; along y it is a whole other row:
//    every access of a wavefront is coalesced.
//  * One thread relaxes one node in registers; the entropy-limited omega
//    (eq. variableOmegaProblem) is solved there, no memory traffic.
//  * Composed step (eq. splittingToUse with eq. basicBrickSplitting): 18 passes
//    "shift, relax" with shifts kappa*(1, 2x7, -1, -4, -1, 2x7) + trailing kappa.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "eslb.h"
#include "eslb_internal.hpp"
#include "eslb_systems.hpp"

using namespace eslb;

namespace {

// ------------------------------------------------------------------ kernels

// Coordinate plus storage shift, both in [0, n): the sum is formed in 32-bit
// unsigned arithmetic, which holds it for every extent up to 2^31 (a signed sum
// would overflow past n = 2^30).
__device__ __forceinline__ unsigned wrap_add(int a, int sh, int n) {
  unsigned s = (unsigned)a + (unsigned)sh;
  if (s >= (unsigned)n) s -= (unsigned)n;
  return s;
}

template <int D>
__device__ __forceinline__ long long storage_index(const Grid& g, int k, int x, int y) {
  if (Lat<D>::axis(k) == 0) return (long long)y * g.nx + wrap_add(x, g.sh[k], g.nx);
  return (long long)wrap_add(y, g.sh[k], g.ny) * g.nx + x;
}

// Planes of at most 2^29 nodes: byte offsets within a plane fit 32 bits, and
// with the plane base wave-uniform the accesses take the scalar-base +
// 32-bit-offset form (no per-lane 64-bit address arithmetic).
constexpr long long kPlane32 = 1ll << 29;

// Largest grid extent per axis.
constexpr int kMaxExtent = (int)((1ll << 31) - (1ll << 16));

template <int D>
__device__ __forceinline__ unsigned storage_offset32(const Grid& g, int k, int x, int y) {
  int xs = x, ys = y;
  if (Lat<D>::axis(k) == 0) {
    xs += g.sh[k];
    if (xs >= g.nx) xs -= g.nx;
  } else {
    ys += g.sh[k];
    if (ys >= g.ny) ys -= g.ny;
  }
  return ((unsigned)ys * (unsigned)g.nx + (unsigned)xs) * 8u;
}

// Base pointers of the q M planes, computed on the host.  Kernel arguments
// live in scalar registers, and as independent pointers (rather than one base
// plus plane multiples, which the compiler folds into per-lane 64-bit adds)
// each access keeps the scalar-base + 32-bit-offset form.
struct Planes {
  double* p[16];
};

__device__ __forceinline__ double& plane_at(double* base, unsigned byte_off) {
  return *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + byte_off);
}

__device__ __forceinline__ void record_flags(DevStats* st, unsigned flags) {
  if (flags) {
    atomicOr(&st->flags, flags);
    if (flags & FLAG_FALLBACK) atomicAdd(&st->n_fallback, 1ull);
  }
}

__device__ __forceinline__ void record_omega(DevStats* st, bool act, double om) {
  double mn = act ? om : INFINITY, mx = act ? om : -INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  if (__lane_id() == 0 && mn <= mx) {
    atomicMin(&st->om_min_bits, (unsigned long long)__double_as_longlong(mn));
    atomicMax(&st->om_max_bits, (unsigned long long)__double_as_longlong(mx));
  }
}

// The relaxation of one node in the stage kernel: through this thread's LDS
// slots for systems with S::kLdsD (the launch gives lds_slots<S>() doubles per
// thread of dynamic LDS), in registers otherwise.
template <class S>
__device__ __forceinline__ double stage_relax(double (&f)[S::Q][S::M], int mode, const Phys& P, unsigned& flags,
                                              double& lam) {
  if constexpr (S::kLdsD) {
    // blocks of kLdsStride threads (stage_shape), each thread its own slots
    extern __shared__ double stage_lds[];
    return relax_node_lds<S>(f, mode, P, flags, lam, stage_lds + threadIdx.y * blockDim.x + threadIdx.x);
  } else {
    return relax_node<S>(f, mode, P, flags, lam);
  }
}

template <class S>
constexpr size_t stage_lds_bytes() {
  return S::kLdsD ? (size_t)kLdsStride * lds_slots<S>() * sizeof(double) : 0;
}

// One relaxation pass (the shift that precedes it is in g.sh).  Off32: planes
// of at most kPlane32 nodes (32-bit byte offsets); otherwise 64-bit indices.
// Rec (the adjoint's recomputation): the pass input is also written to the
// planes rec (same storage layout and offsets) and lambda to lamr (logical node
// order; NaN where the root search fell back), so the adjoint pass needs no
// copy of its input and no root search.
template <class S, int D, bool Off32, bool Rec = false>
// S::kStageBlocks (recording form: S::kRecBlocks) resident blocks of 256 threads
// per CU, i.e. that many waves per SIMD and 512 / that many VGPRs: four for the
// Euler pass and 1D shallow water, three for the Euler recording pass and 2D
// shallow water, two for the 2D scalar systems (see each system)
__global__ __launch_bounds__(256, Rec ? S::kRecBlocks : S::kStageBlocks) void k_stage(Grid g, Planes pl, Phys P, int mode, int track,
                                                               DevStats* st, Planes rec, double* lamr) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int by = g.rev ? (int)(gridDim.y - 1u - blockIdx.y) : (int)blockIdx.y;
  const int y = by * blockDim.y + threadIdx.y;
  const bool act = (x < g.nx) && (y < g.ny);
  unsigned flags = 0;
  double om = 2.0;
  if (act) {
    double f[Q][M];
    bool fin = true;
    if constexpr (Off32) {
      unsigned off[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        off[k] = storage_offset32<D>(g, k, x, y);
#pragma unroll
        for (int m = 0; m < M; ++m) f[k][m] = plane_at(pl.p[k * M + m], off[k]);
      }
      if constexpr (Rec) {
        // records are read back only by the adjoint passes, much later: streaming
        // (non-temporal) stores keep them out of the caches (measured 2% faster)
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) __builtin_nontemporal_store(f[k][m], &plane_at(rec.p[k * M + m], off[k]));
        double lam;
        om = stage_relax<S>(f, mode, P, flags, lam);
        if (mode == 1) __builtin_nontemporal_store(lam, &lamr[(unsigned)y * (unsigned)g.nx + (unsigned)x]);
      } else {
        double lam;
        om = stage_relax<S>(f, mode, P, flags, lam);
      }
      // the offsets enter the stores as 32-bit values of this block, so that each
      // store takes the scalar-base + 32-bit-offset form (carried across the root
      // search, they become 64-bit addresses and one 64-bit add per store)
#pragma unroll
      for (int k = 0; k < Q; ++k) asm volatile("" : "+v"(off[k]));
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          fin &= isfinite(f[k][m]);
          plane_at(pl.p[k * M + m], off[k]) = f[k][m];
        }
    } else {
      long long id[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        id[k] = storage_index<D>(g, k, x, y);
#pragma unroll
        for (int m = 0; m < M; ++m) f[k][m] = g.f[(long long)(k * M + m) * g.plane + id[k]];
      }
      if constexpr (Rec) {
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) rec.p[k * M + m][id[k]] = f[k][m];
        double lam;
        om = stage_relax<S>(f, mode, P, flags, lam);
        if (mode == 1) lamr[(long long)y * g.nx + x] = lam;
      } else {
        double lam;
        om = stage_relax<S>(f, mode, P, flags, lam);
      }
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          fin &= isfinite(f[k][m]);
          g.f[(long long)(k * M + m) * g.plane + id[k]] = f[k][m];
        }
    }
    if (!fin) flags |= FLAG_NAN;
  }
  record_flags(st, flags);
  if (track) record_omega(st, act, om);
}

template <class S, int D>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ u, double* __restrict__ f, long long plane,
                                               int nx, int ny, Phys P, DevStats* st) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const long long i = (long long)y * nx + x;
  double uu[M], feq[Q][M];
#pragma unroll
  for (int m = 0; m < M; ++m) uu[m] = u[(long long)m * plane + i];
  Eq<S>::equilibrium(uu, feq, P);
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) f[(long long)(k * M + m) * plane + i] = feq[k][m];
  typename S::Node c;
  unsigned flags = 0;
  if (!S::prepare(uu, c, P)) flags |= FLAG_INADMISSIBLE;
  else if (!S::subchar(c, P)) flags |= FLAG_SUBCHAR;
  if (flags) atomicOr(&st->flags, flags);
}

template <class S, int D>
__global__ __launch_bounds__(256) void k_moments(Grid g, double* __restrict__ u) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  long long id[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) id[k] = storage_index<D>(g, k, x, y);
  const long long i = (long long)y * g.nx + x;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double acc = g.f[(long long)m * g.plane + id[0]];
#pragma unroll
    for (int k = 1; k < Q; ++k) acc += g.f[(long long)(k * M + m) * g.plane + id[k]];
    u[(long long)m * g.plane + i] = acc;
  }
}

template <class S, int D>
__global__ __launch_bounds__(256) void k_gather(Grid g, double* __restrict__ out) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const long long i = (long long)y * g.nx + x;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const long long id = storage_index<D>(g, k, x, y);
#pragma unroll
    for (int m = 0; m < M; ++m) out[(long long)(k * M + m) * g.plane + i] = g.f[(long long)(k * M + m) * g.plane + id];
  }
}

// Adjoint of one relaxation pass: h = stage input (storage, offsets in gh.sh),
// gbar = cotangent of the stage output in the same storage; overwritten with hbar.
// Taped: lamr holds the forward pass's lambda per node (k_stage with Rec).
template <class S, int D, bool Taped = false>
__global__ __launch_bounds__(256, 2) void k_adjoint_stage(Grid gh, double* __restrict__ gbar, Phys P, int mode,
                                                        DevStats* st, const double* __restrict__ lamr) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= gh.nx || y >= gh.ny) return;
  double u[M], d[Q][M], lam, om;
  bool grad;
  unsigned flags = 0;
  {
    double h[Q][M];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const long long i = storage_index<D>(gh, k, x, y);
#pragma unroll
      for (int m = 0; m < M; ++m) h[k][m] = gh.f[(long long)(k * M + m) * gh.plane + i];
    }
    if constexpr (Taped) {
      const double lr = (mode == 1) ? lamr[(long long)y * gh.nx + x] : 0.0;
      adjoint_taped<S>(h, mode, lr, P, u, d, lam, om, grad);
    } else {
      adjoint_root<S>(h, mode, P, flags, u, d, lam, om, grad);
    }
  }
  // the cotangent is read only once the forward relaxation is known (and the
  // storage indices are rebuilt rather than held through the root iteration)
  long long id[Q];
  double gb[Q][M];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    id[k] = storage_index<D>(gh, k, x, y);
#pragma unroll
    for (int m = 0; m < M; ++m) gb[k][m] = gbar[(long long)(k * M + m) * gh.plane + id[k]];
  }
  adjoint_apply<S>(u, d, lam, om, grad, gb, P);
  bool fin = true;
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      fin &= isfinite(gb[k][m]);
      gbar[(long long)(k * M + m) * gh.plane + id[k]] = gb[k][m];
    }
  if (!fin) flags |= FLAG_NAN;
  if (flags) atomicOr(&st->flags, flags);
}

// Logical layout -> storage (inverse of k_gather).
template <class S, int D>
__global__ __launch_bounds__(256) void k_scatter(Grid g, const double* __restrict__ logical) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const long long i = (long long)y * g.nx + x;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const long long id = storage_index<D>(g, k, x, y);
#pragma unroll
    for (int m = 0; m < M; ++m) g.f[(long long)(k * M + m) * g.plane + id] = logical[(long long)(k * M + m) * g.plane + i];
  }
}

// Adjoint of u = sum_k f_k: fbar_k = ubar for every k (logical layout).
template <class S, int D>
__global__ __launch_bounds__(256) void k_moments_adjoint(const double* __restrict__ ubar, double* __restrict__ fbar,
                                                          long long plane, int nx, int ny) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const long long i = (long long)y * nx + x;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double v = ubar[(long long)m * plane + i];
#pragma unroll
    for (int k = 0; k < Q; ++k) fbar[(long long)(k * M + m) * plane + i] = v;
  }
}

// Adjoint of f = f^eq(u): ubar = sum_k J_k(u)^T fbar_k (logical layout).
template <class S, int D>
__global__ __launch_bounds__(256) void k_init_adjoint(const double* __restrict__ u, const double* __restrict__ fbar,
                                                       double* __restrict__ ubar, long long plane, int nx, int ny,
                                                       Phys P) {
  constexpr int Q = S::Q, M = S::M;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= nx || y >= ny) return;
  const long long i = (long long)y * nx + x;
  double uu[M], yk[Q][M], out[M];
#pragma unroll
  for (int m = 0; m < M; ++m) uu[m] = u[(long long)m * plane + i];
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) yk[k][m] = fbar[(long long)(k * M + m) * plane + i];
  typename S::Node c;
  (void)S::prepare(uu, c, P);
  eq_jacobian_T<S>(c, yk, out, P);
#pragma unroll
  for (int m = 0; m < M; ++m) ubar[(long long)m * plane + i] = out[m];
}

// Whole run in one workgroup for domains whose state fits in LDS: the state is
// loaded once in logical layout, every pass of every step runs on LDS with the
// same offset addressing as k_stage (barriers between passes), and the state is
// written back once with the final offsets.  For small grids where a pass is a
// few microseconds of work and a launch per pass would dominate.
struct RunPlan {
  int npass;
  int trailing;
  int shift[32];
  int op[32];           // 0: relax with the context's omega, 1: projection R_1
  long long o_start[4]; // offsets of the velocities when the run starts
};

template <int D>
__device__ __forceinline__ int lds_index(int k, int x, int y, int nx, int ny, long long o) {
  const int axis = Lat<D>::axis(k);
  const int sign = Lat<D>::sign(k);
  if (axis == 0) {
    long long xs = ((long long)x - sign * o) % nx;
    if (xs < 0) xs += nx;
    return y * nx + (int)xs;
  }
  long long ys = ((long long)y - sign * o) % ny;
  if (ys < 0) ys += ny;
  return (int)ys * nx + x;
}

// Block size: the heavy systems (12-16 populations per node) run 256 threads so
// they keep their registers; the light ones use up to 1024.
template <class S>
constexpr int run_lds_threads() {
  return S::Q * S::M >= 12 ? 256 : 1024;
}

template <class S, int D>
__global__ __launch_bounds__(run_lds_threads<S>()) void k_run_lds(Grid g, Phys P, int mode, RunPlan plan,
                                                                   long long nsteps, DevStats* st) {
  constexpr int Q = S::Q, M = S::M;
  extern __shared__ double lds[];
  const int ncell = g.nx * g.ny;
  // load: logical f_k(x) = storage at x - o_start c_k
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const int x = i % g.nx, y = i / g.nx;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const long long id = storage_index<D>(g, k, x, y);
#pragma unroll
      for (int m = 0; m < M; ++m) lds[(k * M + m) * ncell + i] = g.f[(long long)(k * M + m) * g.plane + id];
    }
  }
  unsigned flags = 0;
  unsigned long long nfall = 0;  // node relaxations of this thread that fell back to omega = 1
  long long o = 0;  // offset of the LDS copy relative to the loaded logical layout
  for (long long step = 0; step < nsteps; ++step) {
    for (int p = 0; p < plan.npass; ++p) {
      o += plan.shift[p];
      Phys Pp = P;
      int md = mode;
      if (plan.op[p]) {
        Pp.omega = 1.0;
        md = 0;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
        const int x = i % g.nx, y = i / g.nx;
        int id[Q];
        double f[Q][M];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          id[k] = lds_index<D>(k, x, y, g.nx, g.ny, o);
#pragma unroll
          for (int m = 0; m < M; ++m) f[k][m] = lds[(k * M + m) * ncell + id[k]];
        }
        unsigned nf = 0;
        relax_node<S>(f, md, Pp, nf);
        flags |= nf;
        nfall += (nf & FLAG_FALLBACK) ? 1ull : 0ull;
#pragma unroll
        for (int k = 0; k < Q; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) {
            if (!isfinite(f[k][m])) flags |= FLAG_NAN;
            lds[(k * M + m) * ncell + id[k]] = f[k][m];
          }
      }
    }
    o += plan.trailing;
  }
  __syncthreads();
  // write back: storage position of logical x after the run is x - (o_start + o) c_k,
  // and the LDS holds it at x - o c_k
  Grid ge = g;
  for (int k = 0; k < Q; ++k) {
    const int axis = (D == 1) ? 0 : (k & 1);
    const int sign = (k < Q / 2) ? 1 : -1;
    const long long n = axis == 0 ? g.nx : g.ny;
    long long sh = (-(long long)sign * (plan.o_start[k] + o)) % n;
    if (sh < 0) sh += n;
    ge.sh[k] = (int)sh;
  }
  for (int i = threadIdx.x; i < ncell; i += blockDim.x) {
    const int x = i % g.nx, y = i / g.nx;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const long long id = storage_index<D>(ge, k, x, y);
      const int li = lds_index<D>(k, x, y, g.nx, g.ny, o);
#pragma unroll
      for (int m = 0; m < M; ++m) g.f[(long long)(k * M + m) * g.plane + id] = lds[(k * M + m) * ncell + li];
    }
  }
  if (flags) {
    atomicOr(&st->flags, flags);
    if (nfall) atomicAdd(&st->n_fallback, nfall);
  }
}

// One composed step of a D1Q2 problem per launch, every pass through LDS.  Block
// b owns the output cells [b L, b L + L) and loads the window of W = L + 2H cells
// around them (H: the step's dependency halo, from the schedule).  Inside the
// window population k of logical cell a - H + j sits at index j - sign_k o after
// the passes have moved it by o cells; pass p relaxes the cells whose two
// populations are still exact (the exact index ranges shrink by the shift at every
// pass and are tracked as block-uniform bounds), and the owned cells are stored in
// the layout of the offsets after the step.  Reads src, writes dst (no overlap:
// neighbouring windows overlap, so the step cannot be done in place).
struct FusedPlan {
  int npass;
  int trailing;
  int shift[32];
  int op[32];   // 0: relax with the context's omega, 1: projection R_1
  int L, H;     // owned cells per block, halo cells on each side
};

// 256 threads and 32 KiB windows: several blocks per CU, so one block's barrier
// waits overlap another's work (measured: 512 threads and 64 KiB windows were
// 15-30% slower on every 1D system).
constexpr int kFusedThreads = 256;
constexpr int kFusedWindowBytes = 32768;

template <class S>
__global__ __launch_bounds__(kFusedThreads, S::kStageBlocks) void k_step_fused_1d(const double* __restrict__ src,
                                                                    double* __restrict__ dst, int nx, int sh_in0,
                                                                    int sh_in1, int sh_out0, int sh_out1, Phys P,
                                                                    int mode, FusedPlan fp, DevStats* st) {
  constexpr int M = S::M;
  extern __shared__ double lds[];
  const int L = fp.L, H = fp.H, W = L + 2 * H;
  const long long a = (long long)blockIdx.x * L;
  const int Lb = (nx - a < L) ? (int)(nx - a) : L;
  const int Wb = Lb + 2 * H;
  for (int j = threadIdx.x; j < Wb; j += blockDim.x) {
    long long x = (a - H + j) % nx;
    if (x < 0) x += nx;
    const unsigned s0 = wrap_add((int)x, sh_in0, nx), s1 = wrap_add((int)x, sh_in1, nx);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      lds[m * W + j] = src[(long long)m * nx + s0];
      lds[(M + m) * W + j] = src[(long long)(M + m) * nx + s1];
    }
  }
  unsigned flags = 0;
  unsigned long long nfall = 0;
  int o = 0;
  int lo0 = 0, hi0 = Wb, lo1 = 0, hi1 = Wb;  // exact index ranges of populations 0 and 1
  for (int p = 0; p < fp.npass; ++p) {
    o += fp.shift[p];
    Phys Pp = P;
    int md = mode;
    if (fp.op[p]) {
      Pp.omega = 1.0;
      md = 0;
    }
    const int rlo = max(lo0 + o, lo1 - o), rhi = min(hi0 + o, hi1 - o);
    __syncthreads();
    for (int j = rlo + (int)threadIdx.x; j < rhi; j += blockDim.x) {
      double f[2][M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        f[0][m] = lds[m * W + j - o];
        f[1][m] = lds[(M + m) * W + j + o];
      }
      unsigned nf = 0;
      relax_node<S>(f, md, Pp, nf);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (!isfinite(f[0][m]) || !isfinite(f[1][m])) nf |= FLAG_NAN;
        lds[m * W + j - o] = f[0][m];
        lds[(M + m) * W + j + o] = f[1][m];
      }
      flags |= nf;
      nfall += (nf & FLAG_FALLBACK) ? 1ull : 0ull;
    }
    lo0 = rlo - o;
    hi0 = rhi - o;
    lo1 = rlo + o;
    hi1 = rhi + o;
  }
  o += fp.trailing;
  __syncthreads();
  for (int t = threadIdx.x; t < Lb; t += blockDim.x) {
    const int x = (int)a + t, j = H + t;
    const unsigned s0 = wrap_add(x, sh_out0, nx), s1 = wrap_add(x, sh_out1, nx);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      dst[(long long)m * nx + s0] = lds[m * W + j - o];
      dst[(long long)(M + m) * nx + s1] = lds[(M + m) * W + j + o];
    }
  }
  if (flags) {
    atomicOr(&st->flags, flags);
    if (nfall) atomicAdd(&st->n_fallback, nfall);
  }
}

// A segment of fixed-omega passes of a D2Q4 problem per launch, every pass through
// LDS: block (bx, by) owns a T x T tile and loads the window of (T + 2H)^2 cells
// around it (H: the segment's dependency halo).  Population k of window cell (i, j)
// sits at (i, j) - sign_k o e_axis(k) once the passes have moved it by o cells; the
// exact index ranges of every population (one rectangle each) shrink by the shift
// at every pass and bound the cells relaxed.  As in the 1D kernel the segment reads
// src and writes dst.  Fixed omega only: no root search, few registers, so the
// block can be 1024 threads at one block per CU (the window takes the LDS).
struct Fused2Plan {
  int npass;
  int trailing;
  int shift[32];
  int op[32];
  int T, H, W;  // owned tile side, halo, window side (LDS planes are W x W)
};

constexpr int kFused2Threads = 1024;

template <class S>
__global__ __launch_bounds__(kFused2Threads) void k_fused_2d(const double* __restrict__ src, double* __restrict__ dst,
                                                            int nx, int ny, int4 sh_in, int4 sh_out, Phys P,
                                                            Fused2Plan fp, DevStats* st) {
  constexpr int Q = 4, M = S::M;
  extern __shared__ double lds[];
  const int T = fp.T, H = fp.H, W = fp.W, WW = fp.W * fp.W;
  const int ax = blockIdx.x * T, ay = blockIdx.y * T;
  const int Lx = min(T, nx - ax), Ly = min(T, ny - ay);
  const int Wx = Lx + 2 * H, Wy = Ly + 2 * H;
  const long long plane = (long long)nx * ny;
  const int shi[4] = {sh_in.x, sh_in.y, sh_in.z, sh_in.w};
  const int sho[4] = {sh_out.x, sh_out.y, sh_out.z, sh_out.w};
  for (int idx = threadIdx.x; idx < Wx * Wy; idx += blockDim.x) {
    const int i = idx % Wx, j = idx / Wx;
    int x = (ax - H + i) % nx, y = (ay - H + j) % ny;
    if (x < 0) x += nx;
    if (y < 0) y += ny;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const unsigned xs = (k & 1) == 0 ? wrap_add(x, shi[k], nx) : (unsigned)x;
      const unsigned ys = (k & 1) == 0 ? (unsigned)y : wrap_add(y, shi[k], ny);
#pragma unroll
      for (int m = 0; m < M; ++m) lds[(k * M + m) * WW + j * W + i] = src[(k * M + m) * plane + (long long)ys * nx + xs];
    }
  }
  unsigned flags = 0;
  int o = 0;
  // exact ranges of the populations, each in its own window coordinates
  int lx[4] = {0, 0, 0, 0}, hx[4] = {Wx, Wx, Wx, Wx}, ly[4] = {0, 0, 0, 0}, hy[4] = {Wy, Wy, Wy, Wy};
  for (int p = 0; p < fp.npass; ++p) {
    o += fp.shift[p];
    // window offset of population k of a node: -sign_k o along its axis
    const int dx[4] = {-o, 0, o, 0}, dy[4] = {0, -o, 0, o};
    int rlx = lx[0] - dx[0], rhx = hx[0] - dx[0], rly = ly[0] - dy[0], rhy = hy[0] - dy[0];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      rlx = max(rlx, lx[k] - dx[k]);
      rhx = min(rhx, hx[k] - dx[k]);
      rly = max(rly, ly[k] - dy[k]);
      rhy = min(rhy, hy[k] - dy[k]);
    }
    Phys Pp = P;
    if (fp.op[p]) Pp.omega = 1.0;
    const int rw = max(rhx - rlx, 0), rh = max(rhy - rly, 0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < rw * rh; idx += blockDim.x) {
      const int i = rlx + idx % rw, j = rly + idx / rw;
      double f[Q][M];
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) f[k][m] = lds[(k * M + m) * WW + (j + dy[k]) * W + (i + dx[k])];
      relax_node_fixed<S>(f, Pp);
#pragma unroll
      for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          if (!isfinite(f[k][m])) flags |= FLAG_NAN;
          lds[(k * M + m) * WW + (j + dy[k]) * W + (i + dx[k])] = f[k][m];
        }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      lx[k] = rlx + dx[k];
      hx[k] = rhx + dx[k];
      ly[k] = rly + dy[k];
      hy[k] = rhy + dy[k];
    }
  }
  o += fp.trailing;
  __syncthreads();
  const int dx[4] = {-o, 0, o, 0}, dy[4] = {0, -o, 0, o};
  for (int idx = threadIdx.x; idx < Lx * Ly; idx += blockDim.x) {
    const int ti = idx % Lx, tj = idx / Lx;
    const int i = H + ti, j = H + tj, x = ax + ti, y = ay + tj;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const unsigned xs = (k & 1) == 0 ? wrap_add(x, sho[k], nx) : (unsigned)x;
      const unsigned ys = (k & 1) == 0 ? (unsigned)y : wrap_add(y, sho[k], ny);
#pragma unroll
      for (int m = 0; m < M; ++m)
        dst[(k * M + m) * plane + (long long)ys * nx + xs] = lds[(k * M + m) * WW + (j + dy[k]) * W + (i + dx[k])];
    }
  }
  if (flags) atomicOr(&st->flags, flags);
}

// Diagnostics, pass 1: per-block partial sums in a fixed tree order.
// Layout of a block's partials: mass[M], micro, macro (NV = M + 2 doubles).
constexpr int kDiagThreads = 256;

template <class S, int D>
__global__ __launch_bounds__(kDiagThreads) void k_diag(Grid g, Phys P, double* partials, DevStats* st) {
  constexpr int Q = S::Q, M = S::M, NV = M + 2;
  __shared__ double red[NV][kDiagThreads];
  const int tid = threadIdx.x;
  const long long ncell = (long long)g.nx * g.ny;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  unsigned long long n_out = 0, n_inad = 0, n_nan = 0;
  for (long long cidx = (long long)blockIdx.x * kDiagThreads + tid; cidx < ncell;
       cidx += (long long)gridDim.x * kDiagThreads) {
    const int x = (int)(cidx % g.nx), y = (int)(cidx / g.nx);
    double f[Q][M], u[M];
    bool fin = true;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const long long id = storage_index<D>(g, k, x, y);
#pragma unroll
      for (int m = 0; m < M; ++m) {
        f[k][m] = g.f[(long long)(k * M + m) * g.plane + id];
        fin &= isfinite(f[k][m]);
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double a = f[0][m];
#pragma unroll
      for (int k = 1; k < Q; ++k) a += f[k][m];
      u[m] = a;
      acc[m] += a;
    }
    if (!fin) { ++n_nan; continue; }
    typename S::Node c;
    if (!S::prepare(u, c, P)) { ++n_inad; continue; }
    double feq[Q][M], d[Q][M];
    Eq<S>::equilibrium(u, feq, P);
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < M; ++m) d[k][m] = f[k][m] - feq[k][m];
    double F = 0.0, dF = 0.0;
    bool unused = false;
    const bool ok = fsum<S>(c, feq, d, 1.0, F, dF, P, -1.0, unused);
    const double Su = S::macro_entropy(c, P);
    acc[M + 1] += Su;
    if (ok) acc[M] += Su + F; else ++n_out;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) red[v][tid] = acc[v];
  __syncthreads();
  for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int v = 0; v < NV; ++v) red[v][tid] += red[v][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) partials[(long long)blockIdx.x * NV + v] = red[v][0];
  }
  if (n_out) atomicAdd(&st->n_outside, n_out);
  if (n_inad) atomicAdd(&st->n_inadmissible, n_inad);
  if (n_nan) atomicAdd(&st->n_nan, n_nan);
}

// Diagnostics, pass 2: one block sums the partials in a fixed order.
__global__ __launch_bounds__(kDiagThreads) void k_diag_final(const double* partials, int nblocks, int nv, double* out) {
  __shared__ double red[kDiagThreads];
  for (int v = 0; v < nv; ++v) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kDiagThreads) a += partials[(long long)b * nv + v];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

__global__ void k_reset(DevStats* st) {
  st->n_fallback = 0;
  st->om_min_bits = 0x7ff0000000000000ull;  // +inf
  st->om_max_bits = 0;                      // +0
  st->flags = 0;
  st->n_outside = 0;
  st->n_inadmissible = 0;
  st->n_nan = 0;
}

__global__ void k_reset_now(DevStats* st) {
  st->n_outside = 0;
  st->n_inadmissible = 0;
  st->n_nan = 0;
}

// Block partials of the diagnostics reduction for the allocation-free entry point
// (eslb_diagnostics_noalloc): at most kDiagMaxBlocks blocks of M + 2 <= 6 values.
// One copy per device, held until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int kDiagMaxBlocks = 1024;
constexpr int kScratchDoubles = kDiagMaxBlocks * 6;
static __device__ __align__(256) double scratch[kScratchDoubles];

}  // namespace

// ------------------------------------------------------------------ host side

namespace eslb {

thread_local std::string g_last_error;
void eslb_set_global_error(const std::string& msg) { g_last_error = msg; }

static int set_err(eslb_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

static int hip_check(eslb_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return ESLB_OK;
  return set_err(c, ESLB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of `scratch` on each device, resolved once per device with that
// device current (the array's name is not a device address in host code).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

static hipError_t scratch_address(double** out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

static long long pmod(long long a, long long n) {
  long long r = a % n;
  return r < 0 ? r + n : r;
}

Grid make_grid(const eslb_ctx* c, double* f) {
  Grid g;
  g.f = f;
  g.nx = c->pb.nx;
  g.ny = c->pb.ny;
  g.rev = 0;
  g.plane = (long long)c->pb.nx * c->pb.ny;
  for (int k = 0; k < 4; ++k) g.sh[k] = 0;
  for (int k = 0; k < c->q; ++k) {
    const int axis = (c->d == 1) ? 0 : (k & 1);
    const int sign = (k < c->q / 2) ? 1 : -1;
    const long long n = axis == 0 ? c->pb.nx : c->pb.ny;
    // logical f_k(x) is stored at x - o_k sign_k along the axis: storage shift -sign*o_k
    g.sh[k] = (int)pmod(-(long long)sign * c->off[k], n);
  }
  return g;
}

void launch_shape(const eslb_ctx* c, dim3& grid, dim3& block) {
  if (c->d == 1) {
    block = dim3(256, 1, 1);
    grid = dim3((unsigned)(((long long)c->pb.nx + 255) / 256), 1, 1);
  } else {
    const int bx = c->pb.nx >= 64 ? 64 : 32;
    const int by = 256 / bx;
    block = dim3(bx, by, 1);
    grid = dim3((unsigned)(((long long)c->pb.nx + bx - 1) / bx), (unsigned)(((long long)c->pb.ny + by - 1) / by), 1);
  }
}

// The stage and adjoint-stage kernels on D2Q4 grids: 128-thread blocks (two
// waves).  Their waves run for very different times (root searches), and a
// smaller block frees its CU slots sooner: 64 x 2 was 1% faster than 64 x 4 on the
// 4096^2 Euler and SW2D passes, 0.7% on the 1024^2 Euler forward + adjoint; 128 x 1
// (one row per block) takes another 1.6% off the Euler pass and 1.3% off the
// forward + adjoint.  D1Q2 keeps 256 threads (smaller blocks measured slower).
void stage_shape(const eslb_ctx* c, dim3& grid, dim3& block) {
  launch_shape(c, grid, block);
  if (c->d == 2) {
    // kLdsStride = 128 threads: 128 x 1 on grids at least 128 wide (a wave's row
    // segment then spans 1 KiB of each plane, and the partially covered 128-B
    // lines at the ends of the x-shifted segments cost half as much: 4096^2 Euler
    // FETCH_SIZE -5.6%, pass -1.6% against 64 x 2), else 64 x 2 or 32 x 4
    const int bx = c->pb.nx >= 128 ? 128 : (c->pb.nx >= 64 ? 64 : 32), by = kLdsStride / bx;
    block = dim3(bx, by, 1);
    grid = dim3((unsigned)(((long long)c->pb.nx + bx - 1) / bx), (unsigned)(((long long)c->pb.ny + by - 1) / by), 1);
  }
}

#define ESLB_DISPATCH(KIND, CALL) ESLB_DISPATCH_KIND(KIND, CALL)

// rec (optional): q*M planes that receive the pass input, and lamr (optional
// with rec; needed for mode 1) one plane for lambda; see k_stage.
int launch_stage(eslb_ctx* c, double* f, int mode, double* rec, double* lamr) {
  Grid g = make_grid(c, f);
  // Every other pass takes the block rows in reverse order, so that it starts on
  // the rows the previous pass ended with, whose lines the memory-side cache
  // (256 MB, an eighth of a 4096^2 Euler state) still holds: 4096^2 Euler,
  // fixed omega 816 -> 762 us per pass, entropic 830 -> 815 us (same box).  Each
  // node's arithmetic does not depend on the order: the same bits.
  g.rev = (int)(c->stage_launches++ & 1u);
  dim3 grid, block;
  stage_shape(c, grid, block);
  const int track = (mode == 1) ? c->track : 0;
  Phys P = c->phys;
  Planes pl{}, rp{};
  for (int i = 0; i < c->q * c->M; ++i) pl.p[i] = f + (long long)i * g.plane;
  if (rec)
    for (int i = 0; i < c->q * c->M; ++i) rp.p[i] = rec + (long long)i * g.plane;
  const bool o32 = g.plane <= kPlane32;
  if (o32 && !rec) {
#define CALL(S, D) hipLaunchKernelGGL((k_stage<S, D, true, false>), grid, block, stage_lds_bytes<S>(), c->stream, g, pl, P, mode, track, c->st, rp, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  } else if (!rec) {
#define CALL(S, D) hipLaunchKernelGGL((k_stage<S, D, false, false>), grid, block, stage_lds_bytes<S>(), c->stream, g, pl, P, mode, track, c->st, rp, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  } else if (o32) {
#define CALL(S, D) hipLaunchKernelGGL((k_stage<S, D, true, true>), grid, block, stage_lds_bytes<S>(), c->stream, g, pl, P, mode, track, c->st, rp, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  } else {
#define CALL(S, D) hipLaunchKernelGGL((k_stage<S, D, false, true>), grid, block, stage_lds_bytes<S>(), c->stream, g, pl, P, mode, track, c->st, rp, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  }
  return hip_check(c, hipGetLastError(), "stage kernel launch");
}

int launch_stage(eslb_ctx* c, double* f, int mode) { return launch_stage(c, f, mode, nullptr, nullptr); }

static int kind_of(const eslb_problem& p, int* d, int* q, int* M) {
  if (p.lattice == ESLB_D1Q2) {
    *d = 1; *q = 2;
    switch (p.system) {
      case ESLB_ADVECTION: *M = 1; return KIND_ADV1;
      case ESLB_BURGERS: *M = 1; return KIND_BUR1;
      case ESLB_SHALLOW_WATER: *M = 2; return KIND_SW1;
      default: return -1;
    }
  }
  if (p.lattice == ESLB_D2Q4) {
    *d = 2; *q = 4;
    switch (p.system) {
      case ESLB_ADVECTION: *M = 1; return KIND_ADV2;
      case ESLB_BURGERS: *M = 1; return KIND_BUR2;
      case ESLB_SHALLOW_WATER: *M = 3; return KIND_SW2;
      case ESLB_EULER: *M = 4; return KIND_EU2;
      default: return -1;
    }
  }
  return -1;
}

int validate_problem(const eslb_problem* p, std::string& why, int* kind, int* d, int* q, int* M) {
  if (!p) { why = "problem is NULL"; return ESLB_ERR_INVALID_ARG; }
  if (p->lattice != ESLB_D1Q2 && p->lattice != ESLB_D2Q4) { why = "unknown lattice"; return ESLB_ERR_INVALID_ARG; }
  if (p->system < ESLB_ADVECTION || p->system > ESLB_EULER) { why = "unknown system"; return ESLB_ERR_INVALID_ARG; }
  const int k = kind_of(*p, d, q, M);
  if (k < 0) { why = "lattice/system combination not supported (Euler needs D2Q4)"; return ESLB_ERR_UNSUPPORTED; }
  *kind = k;
  if (p->nx < 1 || p->ny < 1) { why = "nx and ny must be >= 1"; return ESLB_ERR_INVALID_ARG; }
  if (p->lattice == ESLB_D1Q2 && p->ny != 1) { why = "D1Q2 needs ny == 1"; return ESLB_ERR_INVALID_ARG; }
  if ((long long)p->nx * p->ny > (1ll << 40)) { why = "grid too large"; return ESLB_ERR_INVALID_ARG; }
  // kernels form node coordinates as int from rounded-up grids (up to 1023
  // threads past the extent)
  if (p->nx > kMaxExtent || p->ny > kMaxExtent) { why = "nx and ny must be <= 2^31 - 2^16"; return ESLB_ERR_INVALID_ARG; }
  if (p->kappa < 1) { why = "kappa must be >= 1"; return ESLB_ERR_INVALID_ARG; }
  if (!(p->V > 0.0) || !std::isfinite(p->V)) { why = "V must be > 0"; return ESLB_ERR_INVALID_ARG; }
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) { why = "dx must be > 0"; return ESLB_ERR_INVALID_ARG; }
  if (p->relax != ESLB_OMEGA_FIXED && p->relax != ESLB_OMEGA_ENTROPIC) { why = "unknown relax mode"; return ESLB_ERR_INVALID_ARG; }
  if (p->relax == ESLB_OMEGA_FIXED && !(p->omega > 0.0 && p->omega <= 2.0)) {
    why = "fixed omega must lie in (0, 2]";
    return ESLB_ERR_INVALID_ARG;
  }
  if (p->scheme < 1 || p->scheme > 6) { why = "scheme must be 1..6"; return ESLB_ERR_INVALID_ARG; }
  if (p->reserved != 0) { why = "reserved must be 0"; return ESLB_ERR_INVALID_ARG; }
  if (p->system == ESLB_SHALLOW_WATER && !(p->param[0] > 0.0)) { why = "shallow water needs g > 0"; return ESLB_ERR_INVALID_ARG; }
  if (p->system == ESLB_EULER && !(p->param[0] > 1.0)) { why = "Euler needs gamma > 1"; return ESLB_ERR_INVALID_ARG; }
  return ESLB_OK;
}

Phys make_phys(const eslb_problem& p, int q) {
  Phys P;
  P.V = p.V;
  P.inv2V = 1.0 / (2.0 * p.V);
  P.w = 1.0 / q;
  P.W0 = 2.0 * P.w * p.V;
  P.p0 = p.param[0];
  P.p1 = p.param[1];
  P.p2 = (p.system == ESLB_EULER) ? 1.0 / (p.param[0] - 1.0) : 0.0;
  P.omega = p.omega;
  P.V2 = 2.0 * p.V;
  P.q0 = (p.system == ESLB_EULER) ? -p.V * (p.param[0] + 1.0) / (p.param[0] - 1.0) : 0.0;
  return P;
}

void build_schedule(eslb_ctx* c) {
  // eq. splittingToUse with eq. basicBrickSplitting, consecutive shifts merged
  // (transport moves no data, so merging is only bookkeeping).
  const int k = c->pb.kappa;
  c->passes.clear();
  if (c->pb.scheme == 3) {
    // Scheme III: R_1 after every brick (Sec. 6.1)
    for (int b = 0; b < 9; ++b) {
      const int s = (b == 4) ? -2 * k : k;  // brick psi(dt/6) moves (1,2,1)k, psi(-dt/3) (-2,-4,-2)k
      c->passes.push_back({s, PASS_RELAX});
      c->passes.push_back({2 * s, PASS_RELAX});
      c->passes.push_back({s, PASS_PROJECT});
    }
    c->trailing = 0;
    return;
  }
  if (c->pb.scheme == 4) {
    // standard second-order LB at the same cost (Sec. 3.1, fair comparison): (R T(dt/24))^24
    for (int i = 0; i < 24; ++i) c->passes.push_back({k, PASS_RELAX});
    c->trailing = 0;
    return;
  }
  if (c->pb.scheme == 5) {
    // Scheme (A) of Sec. 6.3: R T(dt), dt = kappa dx / V
    c->passes.push_back({k, PASS_RELAX});
    c->trailing = 0;
    return;
  }
  if (c->pb.scheme == 6) {
    // Scheme (B) of Sec. 6.3: R_1 T(dt/4) R T(dt/2) R T(dt/4), dt = 4 kappa dx / V
    c->passes.push_back({k, PASS_RELAX});
    c->passes.push_back({2 * k, PASS_RELAX});
    c->passes.push_back({k, PASS_PROJECT});
    c->trailing = 0;
    return;
  }
  const int shifts[18] = {1, 2, 2, 2, 2, 2, 2, 2, -1, -4, -1, 2, 2, 2, 2, 2, 2, 2};
  for (int i = 0; i < 18; ++i) c->passes.push_back({shifts[i] * k, PASS_RELAX});
  if (c->pb.scheme == 2) {
    c->passes.push_back({k, PASS_PROJECT});  // Scheme II: R_1 after Phi
    c->trailing = 0;
  } else {
    c->trailing = k;
  }
}

void add_offsets(eslb_ctx* c, long long s) {
  for (int k = 0; k < c->q; ++k) c->off[k] += s;
}

int run_pass(eslb_ctx* c, double* f, int shift, int op) {
  add_offsets(c, shift);
  const int mode = (op == PASS_PROJECT) ? 0 : c->pb.relax;
  if (op == PASS_PROJECT) {
    const double keep = c->phys.omega;
    c->phys.omega = 1.0;
    const int rc = launch_stage(c, f, 0);
    c->phys.omega = keep;
    return rc;
  }
  return launch_stage(c, f, mode);
}


// lamr (optional): the forward pass's lambda plane (launch_stage with rec).
int launch_adjoint_stage(eslb_ctx* c, const double* h, double* gbar, int op, const double* lamr = nullptr) {
  const Grid g = make_grid(c, const_cast<double*>(h));
  dim3 grid, block;
  stage_shape(c, grid, block);
  Phys P = c->phys;
  int mode = c->pb.relax;
  if (op == PASS_PROJECT) {
    P.omega = 1.0;
    mode = 0;
  }
  if (lamr && mode == 1) {
#define CALL(S, D) hipLaunchKernelGGL((k_adjoint_stage<S, D, true>), grid, block, 0, c->stream, g, gbar, P, mode, c->st, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  } else {
#define CALL(S, D) hipLaunchKernelGGL((k_adjoint_stage<S, D, false>), grid, block, 0, c->stream, g, gbar, P, mode, c->st, lamr)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  }
  return hip_check(c, hipGetLastError(), "adjoint stage launch");
}

int launch_layout(eslb_ctx* c, double* storage, const double* logical, bool to_storage) {
  const Grid g = make_grid(c, storage);
  dim3 grid, block;
  launch_shape(c, grid, block);
  if (to_storage) {
#define CALL(S, D) hipLaunchKernelGGL((k_scatter<S, D>), grid, block, 0, c->stream, g, logical)
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  } else {
#define CALL(S, D) hipLaunchKernelGGL((k_gather<S, D>), grid, block, 0, c->stream, g, const_cast<double*>(logical))
    ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  }
  return hip_check(c, hipGetLastError(), "layout kernel launch");
}

long long net_shift(const eslb_ctx* c) {
  long long s = c->trailing;
  for (const Pass& p : c->passes) s += p.shift;
  return s;
}

// Workspace of the reverse sweep (beyond the checkpoints): running state,
// cotangent, and pass records.  Per-step recomputation: one segment's step
// states, one step's stage inputs and lambda planes.  Taped: the stage input and
// lambda plane of every pass of one segment.
size_t sweep_bytes(const eslb_ctx* c, int64_t nsteps, int64_t ck, bool taped) {
  const int64_t lseg = std::min<int64_t>(ck, nsteps);
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  const size_t plane_bytes = (size_t)c->pb.nx * c->pb.ny * sizeof(double), np = c->passes.size();
  const size_t nrec = taped ? (size_t)lseg * np : np;
  return (2 + (taped ? 0 : (size_t)lseg) + nrec) * sb + nrec * plane_bytes;
}

size_t checkpoint_bytes(const eslb_ctx* c, int64_t nsteps, int64_t ck) {
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  return (size_t)((nsteps + ck - 1) / ck) * sb;
}

// Reverse sweep of eslb_adjoint from the checkpoints ckp (states at steps 0, ck,
// 2ck, ... in storage layout); the context's offsets are those of step 0.
int adjoint_sweep(eslb_ctx* c, const double* ckp, int64_t nsteps, int64_t ck, double* fbar, double* wk,
                  bool taped) {
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  const size_t sd = sb / sizeof(double);
  const size_t plane = (size_t)c->pb.nx * c->pb.ny;
  const int64_t nseg = (nsteps + ck - 1) / ck;
  const int64_t lseg = std::min<int64_t>(ck, nsteps);  // steps per segment
  const int npass = (int)c->passes.size();
  double* run = wk;        // running state
  double* cot = run + sd;  // cotangent in storage layout
  double* seg = cot + sd;  // recomputation: lseg step states of one segment
  // pass records: stage inputs and lambda planes, of one step (recomputation)
  // or of every step of a segment (taped)
  const size_t nrec = taped ? (size_t)lseg * npass : (size_t)npass;
  double* stin = taped ? seg : seg + (size_t)lseg * sd;
  double* lamp = stin + nrec * sd;
  long long o0[4];
  for (int k = 0; k < 4; ++k) o0[k] = c->off[k];
  const long long net = net_shift(c);
  long long all_shifts = 0;
  for (int p = 0; p < npass; ++p) all_shifts += c->passes[p].shift;
  auto set_step = [&](int64_t s) {
    for (int k = 0; k < c->q; ++k) c->off[k] = o0[k] + s * net;
  };
  auto copy = [&](double* dst, const double* src) {
    return hip_check(c, hipMemcpyAsync(dst, src, sb, hipMemcpyDeviceToDevice, c->stream), "device copy");
  };
  // the passes of step s on the state f, each recording its input (rec + p sd)
  // and lambda (lam + p plane)
  auto record_step = [&](int64_t s, double* f, double* rec, double* lam) {
    set_step(s);
    int rc = ESLB_OK;
    for (int p = 0; p < npass && rc == ESLB_OK; ++p) {
      add_offsets(c, c->passes[p].shift);
      double* r = rec + (size_t)p * sd;
      double* l = lam + (size_t)p * plane;
      if (c->passes[p].op == PASS_PROJECT) {
        const double keep = c->phys.omega;
        c->phys.omega = 1.0;
        rc = launch_stage(c, f, 0, r, l);
        c->phys.omega = keep;
      } else {
        rc = launch_stage(c, f, c->pb.relax, r, l);
      }
    }
    return rc;
  };
  // the adjoint passes of step s in reverse, from its records
  auto adjoint_step = [&](int64_t s, double* rec, double* lam) {
    set_step(s);
    add_offsets(c, all_shifts);
    int rc = ESLB_OK;
    for (int p = npass - 1; p >= 0 && rc == ESLB_OK; --p) {
      rc = launch_adjoint_stage(c, rec + (size_t)p * sd, cot, c->passes[p].op, lam + (size_t)p * plane);
      add_offsets(c, -c->passes[p].shift);
    }
    return rc;
  };
  // terminal cotangent into storage layout
  set_step(nsteps);
  int rc = launch_layout(c, cot, fbar, true);
  for (int64_t i = nseg - 1; i >= 0 && rc == ESLB_OK; --i) {
    const int64_t s0 = i * ck, s1 = std::min<int64_t>(nsteps, s0 + ck);
    if (taped) {
      rc = copy(run, ckp + (size_t)i * sd);
      for (int64_t s = s0; s < s1 && rc == ESLB_OK; ++s)
        rc = record_step(s, run, stin + (size_t)(s - s0) * npass * sd, lamp + (size_t)(s - s0) * npass * plane);
      for (int64_t s = s1 - 1; s >= s0 && rc == ESLB_OK; --s)
        rc = adjoint_step(s, stin + (size_t)(s - s0) * npass * sd, lamp + (size_t)(s - s0) * npass * plane);
    } else {
      set_step(s0);
      rc = copy(seg, ckp + (size_t)i * sd);
      for (int64_t j = 1; j < s1 - s0 && rc == ESLB_OK; ++j) {
        rc = copy(seg + (size_t)j * sd, seg + (size_t)(j - 1) * sd);
        if (rc == ESLB_OK) rc = eslb_step(c, seg + (size_t)j * sd, 1);
      }
      for (int64_t s = s1 - 1; s >= s0 && rc == ESLB_OK; --s) {
        rc = copy(run, seg + (size_t)(s - s0) * sd);
        if (rc == ESLB_OK) rc = record_step(s, run, stin, lamp);
        if (rc == ESLB_OK) rc = adjoint_step(s, stin, lamp);
      }
    }
  }
  // cotangent of the initial state back to logical layout
  set_step(0);
  if (rc == ESLB_OK) rc = launch_layout(c, cot, fbar, false);
  for (int k = 0; k < 4; ++k) c->off[k] = o0[k];
  return rc;
}

// Whole run in LDS (see k_run_lds); all velocities share one offset history here.
int run_small(eslb_ctx* c, double* f, int64_t nsteps) {
  RunPlan plan;
  plan.npass = (int)c->passes.size();
  plan.trailing = c->trailing;
  for (int p = 0; p < plan.npass; ++p) {
    plan.shift[p] = c->passes[p].shift;
    plan.op[p] = c->passes[p].op == PASS_PROJECT ? 1 : 0;
  }
  const Grid g = make_grid(c, f);
  const long long ncell = (long long)c->pb.nx * c->pb.ny;
  const size_t lds = (size_t)c->q * c->M * ncell * sizeof(double);
  for (int k = 0; k < 4; ++k) plan.o_start[k] = c->off[k];
  Phys P = c->phys;
  const int mode = c->pb.relax;
#define CALL(S, D)                                                                                          \
  hipLaunchKernelGGL((k_run_lds<S, D>), dim3(1),                                                            \
                     dim3((int)std::min<long long>(run_lds_threads<S>(), ((ncell + 63) / 64) * 64)), lds,   \
                     c->stream, g, P, mode, plan, (long long)nsteps, c->st)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  const int rc = hip_check(c, hipGetLastError(), "whole-run kernel launch");
  if (rc == ESLB_OK) add_offsets(c, (long long)nsteps * net_shift(c));
  return rc;
}

// Dependency halo of a run of passes (shifts, then a trailing shift): the
// smallest H for which a window of H extra cells on each side leaves its owned
// cells exact.  The exact index ranges of the two populations of an axis are kept
// as offsets from both window ends ([lo, W + ho), independent of W): each pass
// relaxes the cells whose two populations are exact, and the ranges become that
// set moved back by the populations' offsets.  In 2D it applies to each axis.
int segment_halo(const int* shift, int n, int trailing) {
  int o = 0, lo0 = 0, ho0 = 0, lo1 = 0, ho1 = 0;
  for (int p = 0; p < n; ++p) {
    o += shift[p];
    const int rlo = std::max(lo0 + o, lo1 - o), rho = std::min(ho0 + o, ho1 - o);
    lo0 = rlo - o;
    ho0 = rho - o;
    lo1 = rlo + o;
    ho1 = rho + o;
  }
  o += trailing;
  return std::max({0, lo0 + o, lo1 - o, -o - ho0, o - ho1});
}

// Halo of the fused D1Q2 step: the smallest H for which the owned cells of a
// window are exact after one composed step.
int fused_halo(const eslb_ctx* c) {
  int sh[32];
  const int n = (int)c->passes.size();
  for (int p = 0; p < n; ++p) sh[p] = (int)c->passes[p].shift;
  return segment_halo(sh, n, c->trailing);
}

// Whether eslb_step takes the fused kernel (given a workspace).  ESLB_FUSE_AUTO:
// where it measured faster than the per-pass path -- fixed omega (the per-pass
// path is bound by memory and launches: 3.6-4.4x) and the entropic scalar systems
// (Burgers 2^22: 6%); the entropic shallow-water pass is arithmetic-bound and its
// fused version 4% slower (the barriers between passes), so it stays per pass.
bool fused_active(const eslb_ctx* c) {
  if (c->fuse == ESLB_FUSE_OFF) return false;
  // a small D1Q2 state otherwise runs in one workgroup on one CU; windows of one
  // cell per thread spread it over several CUs (the 1024-cell Burgers run: 3.5x)
  if (c->small_run) return c->d == 1 && c->fused_L_small > 0 && c->pb.nx >= 2 * c->fused_L_small;
  if (c->d == 2) return c->fused_W > 0 && c->pb.relax == ESLB_OMEGA_FIXED;  // D2Q4: fixed omega only
  if (c->fused_L <= 0) return false;
  if (c->fuse == ESLB_FUSE_ALWAYS) return true;
  return c->pb.relax == ESLB_OMEGA_FIXED || c->kind != KIND_SW1;
}


// Fixed-omega D2Q4 steps: the passes of all nsteps steps in order (each step's
// trailing shift folded into the next pass), cut greedily into segments whose
// halo stays within fused_Hmax; a segment of two or more passes is one k_fused_2d
// launch from one buffer to the other, a lone pass runs in place through k_stage.
int run_fused_2d(eslb_ctx* c, double* f, int64_t nsteps) {
  const int npass = (int)c->passes.size();
  const int W = c->fused_W;
  const size_t lds = (size_t)c->q * c->M * W * W * sizeof(double);
  Phys P = c->phys;
  double* buf[2] = {f, c->step_work};
  int cur = 0, rc = ESLB_OK;
  std::vector<int> sh, op;
  sh.reserve(64);
  op.reserve(64);
  long long carry = 0;  // trailing shift of the previous step
  auto flush = [&](int trailing) {
    const int n = (int)sh.size();
    if (n == 0) {
      add_offsets(c, trailing);
      return ESLB_OK;
    }
    int r = ESLB_OK;
    // the trailing shift moves offsets only: leave it out of a segment it would widen
    int seg_trailing = trailing;
    if (n >= 2 && segment_halo(sh.data(), n, trailing) > c->fused_Hmax) seg_trailing = 0;
    if (n == 1 || W - 2 * segment_halo(sh.data(), n, seg_trailing) < 8) {
      for (int p = 0; p < n && r == ESLB_OK; ++p) {
        add_offsets(c, sh[p]);
        const double keep = c->phys.omega;
        if (op[p]) c->phys.omega = 1.0;
        r = launch_stage(c, buf[cur], 0);
        c->phys.omega = keep;
      }
      add_offsets(c, trailing);
    } else {
      Fused2Plan fp;
      fp.npass = n;
      fp.trailing = seg_trailing;
      for (int p = 0; p < n; ++p) {
        fp.shift[p] = sh[p];
        fp.op[p] = op[p];
      }
      fp.H = segment_halo(fp.shift, n, seg_trailing);
      fp.W = W;
      fp.T = W - 2 * fp.H;
      const Grid gi = make_grid(c, buf[cur]);
      long long tot = seg_trailing;
      for (int p = 0; p < n; ++p) tot += sh[p];
      add_offsets(c, tot);
      const Grid go = make_grid(c, buf[1 - cur]);
      const dim3 grid((unsigned)(((long long)c->pb.nx + fp.T - 1) / fp.T),
                      (unsigned)(((long long)c->pb.ny + fp.T - 1) / fp.T));
      const int4 si = make_int4(gi.sh[0], gi.sh[1], gi.sh[2], gi.sh[3]);
      const int4 so = make_int4(go.sh[0], go.sh[1], go.sh[2], go.sh[3]);
#define CALL(S, D) hipLaunchKernelGGL((k_fused_2d<S>), grid, dim3(kFused2Threads), lds, c->stream, buf[cur],      \
                                      buf[1 - cur], c->pb.nx, c->pb.ny, si, so, P, fp, c->st)
      switch (c->kind) {
        case KIND_ADV2: CALL(Advection<2>, 2); break;
        case KIND_BUR2: CALL(Burgers<2>, 2); break;
        case KIND_SW2: CALL(ShallowWater<2>, 2); break;
        case KIND_EU2: CALL(Euler2, 2); break;
        default: break;
      }
#undef CALL
      r = hip_check(c, hipGetLastError(), "fused 2D kernel launch");
      cur = 1 - cur;
      add_offsets(c, trailing - seg_trailing);
    }
    sh.clear();
    op.clear();
    return r;
  };
  for (int64_t s = 0; s < nsteps && rc == ESLB_OK; ++s) {
    for (int p = 0; p < npass && rc == ESLB_OK; ++p) {
      const int shift = (int)(c->passes[p].shift + (p == 0 ? carry : 0));
      const int o = c->passes[p].op == PASS_PROJECT ? 1 : 0;
      sh.push_back(shift);
      op.push_back(o);
      if ((int)sh.size() > 32 || segment_halo(sh.data(), (int)sh.size(), 0) > c->fused_Hmax) {
        sh.pop_back();
        op.pop_back();
        rc = flush(0);
        sh.push_back(shift);
        op.push_back(o);
      }
    }
    carry = c->trailing;
  }
  if (rc == ESLB_OK) rc = flush((int)carry);
  if (rc == ESLB_OK && cur == 1) {
    size_t sb = 0;
    eslb_state_bytes(c, &sb);
    rc = hip_check(c, hipMemcpyAsync(f, c->step_work, sb, hipMemcpyDeviceToDevice, c->stream), "device copy");
  }
  return rc;
}

// Composed steps of a D1Q2 problem, one fused kernel per step, alternating
// between f and the step workspace (a final copy when the count is odd).
int run_fused(eslb_ctx* c, double* f, int64_t nsteps) {
  FusedPlan fp;
  fp.npass = (int)c->passes.size();
  fp.trailing = c->trailing;
  for (int p = 0; p < fp.npass; ++p) {
    fp.shift[p] = (int)c->passes[p].shift;
    fp.op[p] = c->passes[p].op == PASS_PROJECT ? 1 : 0;
  }
  fp.H = c->fused_H;
  fp.L = c->small_run ? c->fused_L_small : c->fused_L;
  const int nx = c->pb.nx;
  const unsigned nblk = (unsigned)(((long long)nx + fp.L - 1) / fp.L);
  const size_t lds = (size_t)2 * c->M * (fp.L + 2 * fp.H) * sizeof(double);
  const long long net = net_shift(c);
  Phys P = c->phys;
  const int mode = c->pb.relax;
  double* buf[2] = {f, c->step_work};
  int cur = 0, rc = ESLB_OK;
  for (int64_t s = 0; s < nsteps && rc == ESLB_OK; ++s) {
    const Grid gi = make_grid(c, buf[cur]);
    add_offsets(c, net);
    const Grid go = make_grid(c, buf[1 - cur]);
#define CALL(S, D)                                                                                            \
  hipLaunchKernelGGL((k_step_fused_1d<S>), dim3(nblk), dim3(kFusedThreads), lds, c->stream, buf[cur],         \
                     buf[1 - cur], nx, gi.sh[0], gi.sh[1], go.sh[0], go.sh[1], P, mode, fp, c->st)
    switch (c->kind) {
      case KIND_ADV1: CALL(Advection<1>, 1); break;
      case KIND_BUR1: CALL(Burgers<1>, 1); break;
      case KIND_SW1: CALL(ShallowWater<1>, 1); break;
      default: break;
    }
#undef CALL
    rc = hip_check(c, hipGetLastError(), "fused step kernel launch");
    cur = 1 - cur;
  }
  if (rc == ESLB_OK && cur == 1) {
    size_t sb = 0;
    eslb_state_bytes(c, &sb);
    rc = hip_check(c, hipMemcpyAsync(f, c->step_work, sb, hipMemcpyDeviceToDevice, c->stream), "device copy");
  }
  return rc;
}

}  // namespace eslb

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* eslb_status_string(int code) {
  switch (code) {
    case ESLB_OK: return "ok";
    case ESLB_ERR_INVALID_ARG: return "invalid argument";
    case ESLB_ERR_UNSUPPORTED: return "unsupported lattice/system";
    case ESLB_ERR_HIP: return "HIP runtime error";
    case ESLB_ERR_NOMEM: return "out of memory";
    case ESLB_ERR_INADMISSIBLE: return "inadmissible state (h, rho or p <= 0)";
    case ESLB_ERR_NAN: return "non-finite value in the state";
    case ESLB_WARN_OMEGA_FALLBACK: return "warning: entropic omega fell back to 1 at some nodes";
    case ESLB_WARN_T_NOT_MULTIPLE: return "warning: T is not a multiple of dt";
    case ESLB_WARN_SUBCHARACTERISTIC: return "warning: sub-characteristic condition violated";
    default: return "unknown status";
  }
}

const char* eslb_last_error(const eslb_ctx* c) { return c ? c->err.c_str() : eslb::g_last_error.c_str(); }

int eslb_create(const eslb_problem* p, void* stream, eslb_ctx** out) {
  if (!out) return ESLB_ERR_INVALID_ARG;
  *out = nullptr;
  std::string why;
  int kind = 0, d = 0, q = 0, M = 0;
  const int rc = validate_problem(p, why, &kind, &d, &q, &M);
  if (rc != ESLB_OK) {
    eslb_set_global_error(why);
    return rc;
  }
  eslb_ctx* c = new eslb_ctx();
  c->pb = *p;
  c->kind = kind;
  c->d = d;
  c->q = q;
  c->M = M;
  c->stream = (hipStream_t)stream;
  for (int k = 0; k < 4; ++k) c->off[k] = 0;
  c->phys = make_phys(*p, q);
  build_schedule(c);
  // whole run in one workgroup's LDS when the state is at most 64 KiB
  c->small_run = ((size_t)q * M * (size_t)p->nx * p->ny * sizeof(double) <= 65536) && c->passes.size() <= 32;
  // fused D1Q2 steps: windows of kFusedWindowBytes of LDS, at least 64 owned cells each
  if (d == 2) {
    // square windows filling the 160 KiB of LDS a block may take; segments keep
    // (W / T)^2 <= 2, i.e. H <= 0.146 W
    int W = (int)std::sqrt(163840.0 / (q * M * sizeof(double)));
    while ((size_t)q * M * W * W * sizeof(double) > 163840) --W;
    c->fused_W = W;
    c->fused_Hmax = std::max(1, (int)(0.146 * W));
  }
  if (d == 1 && c->passes.size() <= 32) {
    const int H = fused_halo(c);
    const int W = kFusedWindowBytes / (2 * M * (int)sizeof(double));
    if (W - 2 * H >= 64) {
      c->fused_H = H;
      c->fused_L = W - 2 * H;
    }
    if (kFusedThreads - 2 * H >= 32) {
      c->fused_H = H;
      c->fused_L_small = kFusedThreads - 2 * H;  // window of one cell per thread
    }
  }
  c->diag_blocks = kDiagMaxBlocks;
  const int nv = M + 2;
  // set-up of the allocation-free diagnostics: the static scratch's address on
  // the current device (a failure surfaces in that entry point, not here)
  (void)scratch_address(&c->scratch);
  hipError_t e = hipMalloc(&c->st, sizeof(DevStats));
  if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * ((size_t)c->diag_blocks * nv + nv));
  if (e != hipSuccess) {
    eslb_set_global_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    if (c->st) (void)hipFree(c->st);
    delete c;
    return ESLB_ERR_NOMEM;
  }
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, c->stream, c->st);
  e = hipGetLastError();
  if (e != hipSuccess) {
    eslb_set_global_error(std::string("reset kernel: ") + hipGetErrorString(e));
    (void)hipFree(c->st);
    (void)hipFree(c->partials);
    delete c;
    return ESLB_ERR_HIP;
  }
  *out = c;
  return ESLB_OK;
}

void eslb_destroy(eslb_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->st) (void)hipFree(c->st);
  if (c->partials) (void)hipFree(c->partials);
  delete c;
}

int eslb_state_bytes(const eslb_ctx* c, size_t* bytes) {
  if (!c || !bytes) return ESLB_ERR_INVALID_ARG;
  *bytes = (size_t)c->q * c->M * (size_t)c->pb.nx * c->pb.ny * sizeof(double);
  return ESLB_OK;
}

int eslb_dims(const eslb_ctx* c, int32_t* M, int32_t* q) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  if (M) *M = c->M;
  if (q) *q = c->q;
  return ESLB_OK;
}

// Delta t of one step: the cells every population moves per step, times dx / V
// (24 kappa dx / V for the fourth-order schemes, Sec. 2.3).
static double step_dt(const eslb_ctx* c) { return (double)net_shift(c) * c->pb.dx / c->pb.V; }

int eslb_dt(const eslb_ctx* c, double* dt) {
  if (!c || !dt) return ESLB_ERR_INVALID_ARG;
  *dt = step_dt(c);
  return ESLB_OK;
}

int eslb_steps_for_time(const eslb_ctx* c, double T, int64_t* n) {
  if (!c || !n || !(T >= 0.0) || !std::isfinite(T)) return ESLB_ERR_INVALID_ARG;
  const double dt = step_dt(c);
  const double r = std::floor(T / dt);
  *n = (int64_t)r;
  return (r * dt == T) ? ESLB_OK : ESLB_WARN_T_NOT_MULTIPLE;
}

int eslb_init_equilibrium(eslb_ctx* c, const double* u, double* f) {
  if (!c || !u || !f) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) c->off[k] = 0;
  dim3 grid, block;
  launch_shape(c, grid, block);
  const long long plane = (long long)c->pb.nx * c->pb.ny;
  const int nx = c->pb.nx, ny = c->pb.ny;
  Phys P = c->phys;
#define CALL(S, D) hipLaunchKernelGGL((k_init<S, D>), grid, block, 0, c->stream, u, f, plane, nx, ny, P, c->st)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  int rc = hip_check(c, hipGetLastError(), "init kernel launch");
  if (rc != ESLB_OK) return rc;
  return eslb_sync_status(c);
}

int eslb_step(eslb_ctx* c, double* f, int64_t nsteps) {
  if (!c || !f || nsteps < 0) return set_err(c, ESLB_ERR_INVALID_ARG, "bad argument to eslb_step");
  const bool fused = fused_active(c) && c->step_work && !c->track;
  if (nsteps > 0 && c->small_run && !c->track && !fused) return run_small(c, f, nsteps);
  if (nsteps > 0 && fused)
    return c->d == 1 ? run_fused(c, f, nsteps) : run_fused_2d(c, f, nsteps);
  for (int64_t s = 0; s < nsteps; ++s) {
    for (const Pass& ps : c->passes) {
      const int rc = run_pass(c, f, ps.shift, ps.op);
      if (rc != ESLB_OK) return rc;
    }
    add_offsets(c, c->trailing);
  }
  return ESLB_OK;
}

int eslb_transport(eslb_ctx* c, int32_t cells) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  add_offsets(c, cells);
  return ESLB_OK;
}

int eslb_relax(eslb_ctx* c, double* f) {
  if (!c || !f) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  return launch_stage(c, f, c->pb.relax);
}

int eslb_project(eslb_ctx* c, double* f) {
  if (!c || !f) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  return run_pass(c, f, 0, PASS_PROJECT);
}

int eslb_moments(eslb_ctx* c, const double* f, double* u) {
  if (!c || !f || !u) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  const Grid g = make_grid(c, const_cast<double*>(f));
  dim3 grid, block;
  launch_shape(c, grid, block);
#define CALL(S, D) hipLaunchKernelGGL((k_moments<S, D>), grid, block, 0, c->stream, g, u)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  return hip_check(c, hipGetLastError(), "moments kernel launch");
}

int eslb_gather(eslb_ctx* c, const double* f, double* out) {
  if (!c || !f || !out) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (f == out) return set_err(c, ESLB_ERR_INVALID_ARG, "eslb_gather: out must not alias f");
  const Grid g = make_grid(c, const_cast<double*>(f));
  dim3 grid, block;
  launch_shape(c, grid, block);
#define CALL(S, D) hipLaunchKernelGGL((k_gather<S, D>), grid, block, 0, c->stream, g, out)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  return hip_check(c, hipGetLastError(), "gather kernel launch");
}

int eslb_get_offsets(const eslb_ctx* c, int64_t* o) {
  if (!c || !o) return ESLB_ERR_INVALID_ARG;
  for (int k = 0; k < c->q; ++k) o[k] = c->off[k];
  return ESLB_OK;
}

int eslb_set_offsets(eslb_ctx* c, const int64_t* o) {
  if (!c || !o) return ESLB_ERR_INVALID_ARG;
  for (int k = 0; k < c->q; ++k) c->off[k] = o[k];
  return ESLB_OK;
}

int eslb_set_step_workspace(eslb_ctx* c, void* work, size_t bytes) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  if (work && bytes < sb) return set_err(c, ESLB_ERR_INVALID_ARG, "step workspace smaller than one state");
  c->step_work = (double*)work;
  c->step_work_bytes = work ? bytes : 0;
  return ESLB_OK;
}

int eslb_set_fusion(eslb_ctx* c, int32_t policy) {
  if (!c || policy < ESLB_FUSE_OFF || policy > ESLB_FUSE_ALWAYS) return ESLB_ERR_INVALID_ARG;
  c->fuse = policy;
  return ESLB_OK;
}

int eslb_fused_step_available(const eslb_ctx* c, int32_t* yes) {
  if (!c || !yes) return ESLB_ERR_INVALID_ARG;
  *yes = fused_active(c) ? 1 : 0;
  return ESLB_OK;
}

int eslb_set_stats(eslb_ctx* c, int32_t on) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  c->track = on ? 1 : 0;
  return ESLB_OK;
}

int eslb_reset_counters(eslb_ctx* c) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, c->stream, c->st);
  return hip_check(c, hipGetLastError(), "reset kernel launch");
}

int eslb_sync_status(eslb_ctx* c) {
  if (!c) return ESLB_ERR_INVALID_ARG;
  int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
  if (rc != ESLB_OK) return rc;
  DevStats h;
  rc = hip_check(c, hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost), "status readback");
  if (rc != ESLB_OK) return rc;
  if (h.flags & FLAG_NAN) return set_err(c, ESLB_ERR_NAN, "non-finite value in the state");
  if (h.flags & FLAG_INADMISSIBLE) return set_err(c, ESLB_ERR_INADMISSIBLE, "inadmissible conserved state");
  if (h.flags & FLAG_FALLBACK) return ESLB_WARN_OMEGA_FALLBACK;
  if (h.flags & FLAG_SUBCHAR) return ESLB_WARN_SUBCHARACTERISTIC;
  return ESLB_OK;
}

int eslb_diagnostics(eslb_ctx* c, const double* f, eslb_diag* out) {
  if (!c || !f || !out) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  const Grid g = make_grid(c, const_cast<double*>(f));
  const long long ncell = (long long)c->pb.nx * c->pb.ny;
  long long nb = (ncell + kDiagThreads - 1) / kDiagThreads;
  if (nb > c->diag_blocks) nb = c->diag_blocks;
  const int nblocks = (int)nb;
  const int nv = c->M + 2;
  // counters of the "now" quantities start from zero (a kernel, not a memset node)
  hipLaunchKernelGGL(k_reset_now, dim3(1), dim3(1), 0, c->stream, c->st);
  int rc = hip_check(c, hipGetLastError(), "reset kernel launch");
  if (rc != ESLB_OK) return rc;
  Phys P = c->phys;
#define CALL(S, D) hipLaunchKernelGGL((k_diag<S, D>), dim3(nblocks), dim3(kDiagThreads), 0, c->stream, g, P, c->partials, c->st)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  rc = hip_check(c, hipGetLastError(), "diagnostics kernel launch");
  if (rc != ESLB_OK) return rc;
  double* fin = c->partials + (size_t)c->diag_blocks * nv;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, c->stream, c->partials, nblocks, nv, fin);
  rc = hip_check(c, hipGetLastError(), "diagnostics final launch");
  if (rc != ESLB_OK) return rc;
  double sums[6];
  DevStats h;
  rc = hip_check(c, hipMemcpyAsync(sums, fin, sizeof(double) * nv, hipMemcpyDeviceToHost, c->stream), "readback");
  if (rc == ESLB_OK) rc = hip_check(c, hipMemcpyAsync(&h, c->st, sizeof(h), hipMemcpyDeviceToHost, c->stream), "readback");
  if (rc == ESLB_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
  if (rc != ESLB_OK) return rc;
  std::memset(out, 0, sizeof(*out));
  for (int m = 0; m < c->M; ++m) out->mass[m] = sums[m];
  out->micro_entropy = sums[c->M];
  out->macro_entropy = sums[c->M + 1];
  double mn, mx;
  std::memcpy(&mn, &h.om_min_bits, sizeof(double));
  std::memcpy(&mx, &h.om_max_bits, sizeof(double));
  out->omega_min = mn;
  out->omega_max = mx;
  out->n_fallback = (int64_t)h.n_fallback;
  out->n_outside = (int64_t)h.n_outside;
  out->n_inadmissible = (int64_t)h.n_inadmissible;
  out->n_nan = (int64_t)h.n_nan;
  return eslb_sync_status(c);
}


int eslb_diagnostics_noalloc(eslb_ctx* c, const double* f, double* sums) {
  if (!c || !f || !sums) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (!c->scratch) {
    // set-up failed at eslb_create (or a context made on another device): resolve now
    const int rc = hip_check(c, scratch_address(&c->scratch), "static scratch address");
    if (rc != ESLB_OK) return rc;
  }
  const Grid g = make_grid(c, const_cast<double*>(f));
  const long long ncell = (long long)c->pb.nx * c->pb.ny;
  long long nb = (ncell + kDiagThreads - 1) / kDiagThreads;
  if (nb > c->diag_blocks) nb = c->diag_blocks;
  const int nblocks = (int)nb;
  const int nv = c->M + 2;
  if ((long long)nblocks * nv > kScratchDoubles)
    return set_err(c, ESLB_ERR_INVALID_ARG, "diagnostics partials exceed the static scratch (" +
                                                std::to_string(kScratchDoubles) + " doubles)");
  // every block writes all nv of its partials, so the scratch needs no clearing
  hipLaunchKernelGGL(k_reset_now, dim3(1), dim3(1), 0, c->stream, c->st);
  int rc = hip_check(c, hipGetLastError(), "reset kernel launch");
  if (rc != ESLB_OK) return rc;
  Phys P = c->phys;
  double* part = c->scratch;
#define CALL(S, D) hipLaunchKernelGGL((k_diag<S, D>), dim3(nblocks), dim3(kDiagThreads), 0, c->stream, g, P, part, c->st)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  rc = hip_check(c, hipGetLastError(), "diagnostics kernel launch");
  if (rc != ESLB_OK) return rc;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, c->stream, part, nblocks, nv, sums);
  return hip_check(c, hipGetLastError(), "diagnostics final launch");
}

int eslb_relax_adjoint(eslb_ctx* c, const double* h, double* gbar) {
  if (!c || !h || !gbar) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (h == gbar) return set_err(c, ESLB_ERR_INVALID_ARG, "eslb_relax_adjoint: gbar must not alias h");
  return launch_adjoint_stage(c, h, gbar, PASS_RELAX);
}

int eslb_moments_adjoint(eslb_ctx* c, const double* ubar, double* fbar) {
  if (!c || !ubar || !fbar) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  dim3 grid, block;
  launch_shape(c, grid, block);
  const long long plane = (long long)c->pb.nx * c->pb.ny;
  const int nx = c->pb.nx, ny = c->pb.ny;
#define CALL(S, D) hipLaunchKernelGGL((k_moments_adjoint<S, D>), grid, block, 0, c->stream, ubar, fbar, plane, nx, ny)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  return hip_check(c, hipGetLastError(), "moments adjoint launch");
}

int eslb_init_adjoint(eslb_ctx* c, const double* u, const double* fbar, double* ubar) {
  if (!c || !u || !fbar || !ubar) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  dim3 grid, block;
  launch_shape(c, grid, block);
  const long long plane = (long long)c->pb.nx * c->pb.ny;
  const int nx = c->pb.nx, ny = c->pb.ny;
  Phys P = c->phys;
#define CALL(S, D) hipLaunchKernelGGL((k_init_adjoint<S, D>), grid, block, 0, c->stream, u, fbar, ubar, plane, nx, ny, P)
  ESLB_DISPATCH(c->kind, CALL)
#undef CALL
  return hip_check(c, hipGetLastError(), "init adjoint launch");
}

int eslb_adjoint_workspace_bytes(const eslb_ctx* c, int64_t nsteps, int64_t ckpt_every, size_t* bytes) {
  if (!c || !bytes || nsteps < 0 || ckpt_every < 1) return ESLB_ERR_INVALID_ARG;
  *bytes = checkpoint_bytes(c, nsteps, ckpt_every) + sweep_bytes(c, nsteps, ckpt_every, false);
  return ESLB_OK;
}

int eslb_adjoint_tape_bytes(const eslb_ctx* c, int64_t nsteps, int64_t ckpt_every, size_t* bytes) {
  if (!c || !bytes || nsteps < 0 || ckpt_every < 1) return ESLB_ERR_INVALID_ARG;
  *bytes = checkpoint_bytes(c, nsteps, ckpt_every) + sweep_bytes(c, nsteps, ckpt_every, true);
  return ESLB_OK;
}

int eslb_checkpoint_bytes(const eslb_ctx* c, int64_t nsteps, int64_t ckpt_every, size_t* bytes) {
  if (!c || !bytes || nsteps < 0 || ckpt_every < 1) return ESLB_ERR_INVALID_ARG;
  *bytes = checkpoint_bytes(c, nsteps, ckpt_every);
  return ESLB_OK;
}

int eslb_step_checkpointed(eslb_ctx* c, double* f, int64_t nsteps, int64_t ck, double* ckpt) {
  if (!c || !f || !ckpt) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (nsteps < 0 || ck < 1) return set_err(c, ESLB_ERR_INVALID_ARG, "nsteps must be >= 0 and ckpt_every >= 1");
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  int rc = ESLB_OK;
  for (int64_t s = 0; s < nsteps && rc == ESLB_OK; s += ck) {
    rc = hip_check(c, hipMemcpyAsync(ckpt + (size_t)(s / ck) * (sb / sizeof(double)), f, sb,
                                     hipMemcpyDeviceToDevice, c->stream), "device copy");
    if (rc == ESLB_OK) rc = eslb_step(c, f, std::min<int64_t>(ck, nsteps - s));
  }
  return rc;
}

int eslb_adjoint_checkpointed(eslb_ctx* c, const double* ckpt, int64_t nsteps, int64_t ck, double* fbar,
                              void* work, size_t work_bytes) {
  if (!c || !ckpt || !fbar || !work) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (nsteps < 0 || ck < 1) return set_err(c, ESLB_ERR_INVALID_ARG, "nsteps must be >= 0 and ckpt_every >= 1");
  if (work_bytes < sweep_bytes(c, nsteps, ck, false))
    return set_err(c, ESLB_ERR_INVALID_ARG, "adjoint workspace too small");
  const bool taped = work_bytes >= sweep_bytes(c, nsteps, ck, true);
  return adjoint_sweep(c, ckpt, nsteps, ck, fbar, (double*)work, taped);
}

int eslb_adjoint(eslb_ctx* c, const double* f0, int64_t nsteps, int64_t ck, double* fbar, void* work,
                 size_t work_bytes) {
  if (!c || !f0 || !fbar || !work) return set_err(c, ESLB_ERR_INVALID_ARG, "NULL argument");
  if (nsteps < 0 || ck < 1) return set_err(c, ESLB_ERR_INVALID_ARG, "nsteps must be >= 0 and ckpt_every >= 1");
  const size_t cb = checkpoint_bytes(c, nsteps, ck);
  if (work_bytes < cb + sweep_bytes(c, nsteps, ck, false))
    return set_err(c, ESLB_ERR_INVALID_ARG, "adjoint workspace too small");
  // with room for a whole segment's pass records, the segment is recomputed
  // once, recording as it goes; otherwise its step states are recomputed and
  // each step is run once more, recording, just before its adjoint passes
  const bool taped = work_bytes >= cb + sweep_bytes(c, nsteps, ck, true);
  double* ckp = (double*)work;
  double* wk = ckp + cb / sizeof(double);
  size_t sb = 0;
  eslb_state_bytes(c, &sb);
  long long o0[4];
  for (int k = 0; k < 4; ++k) o0[k] = c->off[k];
  // forward sweep from a copy of f0, keeping a checkpoint every ck steps
  int rc = hip_check(c, hipMemcpyAsync(wk, f0, sb, hipMemcpyDeviceToDevice, c->stream), "device copy");
  if (rc == ESLB_OK) rc = eslb_step_checkpointed(c, wk, nsteps, ck, ckp);
  for (int k = 0; k < 4; ++k) c->off[k] = o0[k];
  if (rc != ESLB_OK) return rc;
  return adjoint_sweep(c, ckp, nsteps, ck, fbar, wk, taped);
}

}  // extern "C"
