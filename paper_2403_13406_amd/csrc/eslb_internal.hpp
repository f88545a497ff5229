// Host/device data shared by the translation units of libeslb.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "eslb.h"
#include "eslb_systems.hpp"

namespace eslb {

// Device-side status block (one per context).
struct DevStats {
  unsigned long long n_fallback;   // node relaxations that used omega = 1 (no entropic root)
  unsigned long long om_min_bits;  // bit pattern of the smallest omega (omega > 0)
  unsigned long long om_max_bits;  // bit pattern of the largest omega
  unsigned int flags;              // FLAG_* (sticky)
  unsigned int pad;
  unsigned long long n_outside;    // diagnostics: nodes outside the convexity domain
  unsigned long long n_inadmissible;
  unsigned long long n_nan;
};

// One state as seen by a kernel: planes and per-velocity storage shifts.
struct Grid {
  double* f;
  long long plane;  // nx * ny
  int nx, ny;
  int sh[4];        // logical node x of velocity k is stored at x + sh[k] (mod n) along its axis
  int rev;          // stage passes: block rows taken in reverse order (see launch_stage)
};

enum Kind { KIND_ADV1, KIND_ADV2, KIND_BUR1, KIND_BUR2, KIND_SW1, KIND_SW2, KIND_EU2 };
enum PassOp { PASS_RELAX = 0, PASS_PROJECT = 1 };
struct Pass {
  int shift;  // cells moved by the transport that precedes the relaxation
  int op;     // PASS_RELAX (context's omega) or PASS_PROJECT (R_1)
};

void eslb_set_global_error(const std::string& msg);

}  // namespace eslb

struct eslb_ctx;

namespace eslb {
// shared host helpers (defined in eslb.hip)
int validate_problem(const eslb_problem* p, std::string& why, int* kind, int* d, int* q, int* M);
Phys make_phys(const eslb_problem& p, int q);
long long net_shift(const eslb_ctx* c);
}  // namespace eslb

// Calls CALL(SystemType, D) for the system kind of a context.
#define ESLB_DISPATCH_KIND(KIND, CALL)                 \
  switch (KIND) {                                      \
    case eslb::KIND_ADV1: CALL(eslb::Advection<1>, 1); break;    \
    case eslb::KIND_ADV2: CALL(eslb::Advection<2>, 2); break;    \
    case eslb::KIND_BUR1: CALL(eslb::Burgers<1>, 1); break;      \
    case eslb::KIND_BUR2: CALL(eslb::Burgers<2>, 2); break;      \
    case eslb::KIND_SW1: CALL(eslb::ShallowWater<1>, 1); break;  \
    case eslb::KIND_SW2: CALL(eslb::ShallowWater<2>, 2); break;  \
    case eslb::KIND_EU2: CALL(eslb::Euler2, 2); break;           \
    default: break;                                    \
  }

struct eslb_ctx {
  eslb_problem pb;
  int kind = 0, d = 1, q = 2, M = 1;
  hipStream_t stream = nullptr;
  long long off[4] = {0, 0, 0, 0};  // logical offsets o_k (cells travelled along V_k / V)
  eslb::Phys phys;
  std::vector<eslb::Pass> passes;   // one composed step
  int trailing = 0;                 // shift after the last pass of a step
  eslb::DevStats* st = nullptr;
  double* partials = nullptr;
  int diag_blocks = 0;
  double* scratch = nullptr;     // device address of the static diagnostics scratch on this context's device
  int track = 0;
  unsigned stage_launches = 0;  // parity of the row order of the next stage pass
  bool small_run = false;  // whole run in one workgroup's LDS (small states)
  int fused_L = 0, fused_H = 0;  // fused D1Q2 step: owned cells per block, halo (0: not available)
  int fused_L_small = 0;         // owned cells per block for states of one workgroup (one cell per thread)
  int fuse = ESLB_FUSE_AUTO;     // eslb_set_fusion policy
  int fused_W = 0, fused_Hmax = 0;  // fused D2Q4 fixed-omega segments: window side, largest halo
  double* step_work = nullptr;   // caller-owned workspace of one state for the fused steps
  size_t step_work_bytes = 0;
  std::string err;
};
