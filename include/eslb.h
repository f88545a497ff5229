/*
 * eslb — fourth-order entropy-stable lattice Boltzmann time loop on gfx950 (MI355X).
 *
 * C ABI of libeslb.so.  Method: Bellotti, Helluy, Navoret, "Fourth-order
 * entropy-stable lattice Boltzmann schemes for hyperbolic systems"
 * (arXiv 2403.13406).  Every entry point cites the passage that defines what it
 * computes.
 *
 * Conventions shared by all calls
 * -------------------------------
 *  - Precision: every value is IEEE binary64.
 *  - Pointers named *_dev are device pointers (HIP global memory) owned by the
 *    caller; the library never frees them and never keeps them after the call
 *    returns.  The library owns only its context, a small device block of status
 *    counters and reduction scratch, and (batch) a descriptor table.
 *  - Distribution layout ("state"): q*M planes of nx*ny doubles, plane
 *    p = k*M + m (k the discrete velocity, m the conserved component), x fastest
 *    inside a plane.  Velocity order: D1Q2 (+, -) (Sec. 1.2.1); D2Q4
 *    (+x, +y, -x, -y) (Sec. 1.2.2).  Conserved-moment arrays u hold M planes of
 *    nx*ny doubles in the same order as the system's variables.
 *  - Transport (eq. transportPhase) moves no data: the context keeps one integer
 *    offset o_k per velocity (cells travelled along V_k/V), and logical
 *    f_k(x) lives at storage position x - o_k (V_k/V), periodic.  f_dev alone is
 *    therefore not the logical state; read it with eslb_moments / eslb_gather,
 *    or save the offsets with eslb_get_offsets.
 *  - Streams: device work is enqueued asynchronously on the stream given to
 *    eslb_create (NULL = the null stream) unless a call says it synchronises.
 *  - Return codes: 0 = ESLB_OK, negative = error (nothing or only part of the
 *    work was done; eslb_last_error has the message), positive = warning (the
 *    work was done).  Device-side conditions (inadmissible state, NaN, omega
 *    fallbacks) are sticky in a device status word and are reported by the next
 *    synchronising call (eslb_sync_status, eslb_diagnostics, eslb_init_equilibrium).
 *  - Threading: a context must not be used from two threads at once.
 */
#ifndef ESLB_H
#define ESLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Lattices DdQq^M (Sec. 1.2.1 and 1.2.2). */
#define ESLB_D1Q2 1
#define ESLB_D2Q4 2

/* Target systems (Sec. 1.1): examples of Sec. 1.2, 2D Burgers of Sec. 3.3,
 * Euler of Sec. 6.3.  M = 1 (advection, Burgers), d+1 (shallow water),
 * d+2 (Euler, D2Q4 only). */
#define ESLB_ADVECTION 0     /* phi^j = a_j u,        param = {a_x, a_y}          */
#define ESLB_BURGERS 1       /* phi^j = b_j u^2 / 2,  param = {b_x, b_y}          */
#define ESLB_SHALLOW_WATER 2 /* (h, hu[, hv]),        param = {g}                 */
#define ESLB_EULER 3         /* (rho, rho u, rho v, E), param = {gamma}           */

/* Relaxation parameter (eq. relaxationDiscretizationOmega, eq. variableOmegaProblem). */
#define ESLB_OMEGA_FIXED 0    /* omega = problem.omega at every node (2 in Sec. 2-3) */
#define ESLB_OMEGA_ENTROPIC 1 /* per-node omega with Sigma(R_omega f) = Sigma(f)    */

/* Status codes. */
#define ESLB_OK 0
#define ESLB_ERR_INVALID_ARG (-1)
#define ESLB_ERR_UNSUPPORTED (-2)
#define ESLB_ERR_HIP (-3)
#define ESLB_ERR_NOMEM (-4)
#define ESLB_ERR_INADMISSIBLE (-6) /* h <= 0, rho <= 0 or p <= 0 in some u            */
#define ESLB_ERR_NAN (-7)          /* a non-finite value appeared in the state        */
#define ESLB_WARN_OMEGA_FALLBACK 1 /* some node had no entropic root: omega = 1 used  */
#define ESLB_WARN_T_NOT_MULTIPLE 2 /* T is not a multiple of Delta t (floor applied)  */
#define ESLB_WARN_SUBCHARACTERISTIC 3 /* V violates the convexity condition somewhere */

/* Problem statement (Sec. 1.1-1.2, Sec. 2.3): lattice, system with its flux
 * parameters, grid, kinetic velocity V, space step dx, kappa (cells moved by the
 * shortest transport T(Delta t / 24); 1 in the paper), relaxation choice and
 * composition variant. */
typedef struct eslb_problem {
  int32_t lattice;   /* ESLB_D1Q2 or ESLB_D2Q4                                   */
  int32_t system;    /* ESLB_ADVECTION .. ESLB_EULER                             */
  int32_t nx, ny;    /* grid; ny must be 1 for D1Q2; periodic in every direction;
                        1 <= nx, ny <= 2^31 - 2^16 and nx * ny <= 2^40        */
  int32_t kappa;     /* >= 1                                                     */
  int32_t relax;     /* ESLB_OMEGA_FIXED or ESLB_OMEGA_ENTROPIC                  */
  int32_t scheme;    /* 1: Phi of eq. splittingToUse (Scheme I); 2, 3: Schemes II
                        and III of Sec. 6.1 (projections R_1 added); comparison
                        schedules: 4: standard LB (R T(dt/24))^24 (Sec. 3.1);
                        5: Scheme (A) R T(dt), dt = kappa dx/V; 6: Scheme (B)
                        R_1 T(dt/4) R T(dt/2) R T(dt/4), dt = 4 kappa dx/V (Sec. 6.3) */
  int32_t reserved;  /* must be 0                                                */
  double V;          /* kinetic velocity, > 0                                    */
  double dx;         /* space step, > 0                                          */
  double omega;      /* used when relax == ESLB_OMEGA_FIXED, in (0, 2]           */
  double param[4];   /* system parameters, see the system constants above       */
} eslb_problem;

/* Synchronous diagnostics of one state (Sec. 4). */
typedef struct eslb_diag {
  double mass[4];        /* sum_x u_m, m < M                                       */
  double micro_entropy;  /* sum_x Sigma(f) = sum_x sum_k s_k(f_k)                  */
  double macro_entropy;  /* sum_x S(u)                                             */
  double omega_min;      /* over entropic relaxations since the last counter reset */
  double omega_max;      /*   (only tracked after eslb_set_stats(ctx, 1))          */
  int64_t n_fallback;    /* node relaxations that fell back to omega = 1 since reset */
  int64_t n_outside;     /* nodes whose populations are outside the convexity domain */
  int64_t n_inadmissible;/* nodes with inadmissible u (now)                        */
  int64_t n_nan;         /* nodes with a non-finite population (now)               */
} eslb_diag;

typedef struct eslb_ctx eslb_ctx;

/* Create a context for one problem (validates it; allocates only the small
 * status/reduction block).  stream: a hipStream_t, or NULL.  On success *out is
 * set; destroy it with eslb_destroy. */
int eslb_create(const eslb_problem* problem, void* stream, eslb_ctx** out);
void eslb_destroy(eslb_ctx* ctx);

/* q * M * nx * ny * 8: bytes of one state. */
int eslb_state_bytes(const eslb_ctx* ctx, size_t* bytes);
/* Number of conserved components M and of velocities q. */
int eslb_dims(const eslb_ctx* ctx, int32_t* M, int32_t* q);

/* Delta t of one step = (cells moved per step) dx / V: 24 kappa dx / V for
 * schemes 1-4 (Sec. 2.3), kappa dx / V for 5, 4 kappa dx / V for 6. */
int eslb_dt(const eslb_ctx* ctx, double* dt);
/* n = floor(T / Delta t) in binary64 (the paper leaves this open); returns
 * ESLB_WARN_T_NOT_MULTIPLE when n * Delta t != T. */
int eslb_steps_for_time(const eslb_ctx* ctx, double T, int64_t* n);

/* f_k = f_k^eq(u) at every node (initial data at equilibrium, Sec. 3.1) and
 * offsets reset to 0.  u_dev: M planes (read); f_dev: q*M planes (written).
 * Synchronises; returns ESLB_ERR_INADMISSIBLE if some u is inadmissible and
 * ESLB_WARN_SUBCHARACTERISTIC if V violates the convexity condition somewhere. */
int eslb_init_equilibrium(eslb_ctx* ctx, const double* u_dev, double* f_dev);

/* Advance nsteps >= 0 composed steps Phi(Delta t) in place (eq. splittingToUse,
 * eq. basicBrickSplitting; Schemes II/III of Sec. 6.1 when selected): per step
 * 18 passes "shift, relax" with shifts kappa * (1, 2 x7, -1, -4, -1, 2 x7) and a
 * trailing shift of kappa.  Asynchronous. */
int eslb_step(eslb_ctx* ctx, double* f_dev, int64_t nsteps);
/* Optional workspace for eslb_step: work_dev, a caller-owned device buffer of at
 * least eslb_state_bytes bytes that aliases no state.  With it (and omega
 * statistics off) eslb_step fuses passes through LDS: on D1Q2 each composed step
 * is one kernel (a window of cells with the step's dependency halo per block); on
 * D2Q4 with fixed omega runs of passes whose halo fits a square window are one
 * kernel each.  A fused kernel reads the state from one buffer and writes the other
 * (neighbouring windows overlap, so not in place); f_dev holds the result on
 * return (one copy when the number of fused launches is odd).  Same bits as the
 * per-pass path.  work_dev = NULL detaches it; the workspace must stay allocated
 * while attached. */
int eslb_set_step_workspace(eslb_ctx* ctx, void* work_dev, size_t bytes);
/* When eslb_step takes the fused kernels (given the workspace): ESLB_FUSE_OFF
 * never; ESLB_FUSE_AUTO (default) where they are the faster path -- fixed omega,
 * and on D1Q2 also entropic omega for the scalar systems (the entropic
 * shallow-water and 2D passes are arithmetic-bound and stay one per launch);
 * ESLB_FUSE_ALWAYS for every D1Q2 problem larger than the single-workgroup case
 * (D2Q4: fixed omega only).  Results are the same bits either way. */
enum { ESLB_FUSE_OFF = 0, ESLB_FUSE_AUTO = 1, ESLB_FUSE_ALWAYS = 2 };
int eslb_set_fusion(eslb_ctx* ctx, int32_t policy);
/* *yes = 1 when eslb_step takes the fused kernel under the current policy once a
 * workspace is attached. */
int eslb_fused_step_available(const eslb_ctx* ctx, int32_t* yes);

/* One transport T(cells) (eq. transportPhase): offsets only, no device work. */
int eslb_transport(eslb_ctx* ctx, int32_t cells);
/* One relaxation pass R_omega at every node with the context's omega choice
 * (eq. relaxationDiscretizationOmega / eq. variableOmegaProblem).  Asynchronous. */
int eslb_relax(eslb_ctx* ctx, double* f_dev);
/* One projection R_1 on the equilibrium (Sec. 6.1).  Asynchronous. */
int eslb_project(eslb_ctx* ctx, double* f_dev);

/* u = sum_k f_k at every logical node (Sec. 1.2), offsets applied.
 * f_dev: q*M planes (read); u_dev: M planes (written).  Asynchronous. */
int eslb_moments(eslb_ctx* ctx, const double* f_dev, double* u_dev);
/* The logical distributions (offsets applied) copied to out_dev (q*M planes, must
 * not alias f_dev): out_dev is the state with all offsets 0.  Asynchronous. */
int eslb_gather(eslb_ctx* ctx, const double* f_dev, double* out_dev);

/* Offsets o_k (q entries, cells travelled along V_k / V). */
int eslb_get_offsets(const eslb_ctx* ctx, int64_t* offsets);
int eslb_set_offsets(eslb_ctx* ctx, const int64_t* offsets);

/* Synchronous diagnostics (see eslb_diag).  Returns the sticky status. */
int eslb_diagnostics(eslb_ctx* ctx, const double* f_dev, eslb_diag* out);
/* Allocation-free variant of eslb_diagnostics, for callers that cannot allocate
 * device memory or synchronise: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Enqueues on the context's stream the
 * same two reduction kernels and writes their sums, in the order
 * mass[0..M-1], micro entropy, macro entropy (M + 2 doubles, the values
 * eslb_diagnostics returns in those fields, to the bit), to sums_dev, a
 * caller-owned device buffer of at least M + 2 doubles.  No allocation, copy,
 * memset or synchronisation: the per-block partial sums (at most 1024 blocks of
 * M + 2 values) live in a library-owned static device array of 6144 doubles
 * (48 KiB per device, held until the process ends).  Every call on a device
 * shares that device's array: calls that overlap in time on one device race
 * (order them, e.g. on one stream).  The nodes outside the convexity domain,
 * inadmissible and non-finite are counted into the context's status block as by
 * eslb_diagnostics; read them with eslb_diagnostics or the sticky status with
 * eslb_sync_status.  Returns ESLB_ERR_INVALID_ARG for NULL arguments,
 * ESLB_ERR_HIP if a launch fails or the array's address cannot be resolved on
 * the current device. */
int eslb_diagnostics_noalloc(eslb_ctx* ctx, const double* f_dev, double* sums_dev);
/* Track omega min/max in every entropic pass (costs a few atomics per block). */
int eslb_set_stats(eslb_ctx* ctx, int32_t on);
/* Zero the device counters and the sticky status.  Asynchronous. */
int eslb_reset_counters(eslb_ctx* ctx);
/* Synchronise the stream and return the sticky status. */
int eslb_sync_status(eslb_ctx* ctx);

/* ---------------------------------------------------------------- adjoint
 * Reverse-mode derivative of the time loop (not in the paper: the derivative of
 * its scheme).  One relaxation maps the stage input h to
 * g = (1-omega) h + omega f^eq(sum h); its adjoint maps gbar to
 *   hbar_j = (1-omega) gbar_j + omega sum_k J_k^T gbar_k
 *            + grad_{h_j} omega * sum_k (f^eq_k - h_k) . gbar_k,
 * with grad omega from the implicit function theorem on eq. variableOmegaProblem
 * (zero term for fixed omega).  The adjoint of a transport T(s) is T(-s), which
 * is offset bookkeeping only. */

/* Adjoint of one eslb_relax pass at the current offsets: h_dev is the pass input
 * (q*M planes, storage layout, read), gbar_dev the cotangent of its output in the
 * same storage layout, overwritten with the cotangent of h.  Must not alias.
 * Asynchronous. */
int eslb_relax_adjoint(eslb_ctx* ctx, const double* h_dev, double* gbar_dev);
/* Adjoint of eslb_moments: fbar_k = ubar for every k (logical layout, offsets 0).
 * ubar_dev: M planes (read); fbar_dev: q*M planes (written).  Asynchronous. */
int eslb_moments_adjoint(eslb_ctx* ctx, const double* ubar_dev, double* fbar_dev);
/* Adjoint of eslb_init_equilibrium: ubar = sum_k (d f_k^eq / du)(u)^T fbar_k.
 * u_dev, ubar_dev: M planes; fbar_dev: q*M planes, logical layout.  Asynchronous. */
int eslb_init_adjoint(eslb_ctx* ctx, const double* u_dev, const double* fbar_dev, double* ubar_dev);
/* Device bytes eslb_adjoint needs for (nsteps, ckpt_every), with L =
 * min(ckpt_every, nsteps) steps per segment and P = passes per step:
 * (ceil(nsteps/ckpt_every) + 2 + L + P) states plus P planes of nx*ny doubles
 * (each pass's lambda). */
int eslb_adjoint_workspace_bytes(const eslb_ctx* ctx, int64_t nsteps, int64_t ckpt_every, size_t* bytes);
/* Device bytes with which eslb_adjoint records a whole segment at once:
 * (ceil(nsteps/ckpt_every) + 2 + L P) states plus L P lambda planes (L, P as
 * above).  Given at least this much workspace, eslb_adjoint recomputes every
 * step once instead of twice; the result is the same to the bit. */
int eslb_adjoint_tape_bytes(const eslb_ctx* ctx, int64_t nsteps, int64_t ckpt_every, size_t* bytes);
/* Cotangent of the initial distributions through nsteps composed steps.
 * f0_dev: the forward initial state in storage layout with the context's current
 * offsets (read only).  fbar_dev: on entry the cotangent of the state after
 * nsteps steps, on return the cotangent of f0; both in logical layout (offsets
 * applied, as eslb_gather returns).  work_dev: caller-owned device workspace of at
 * least eslb_adjoint_workspace_bytes bytes.  Checkpoints every ckpt_every steps;
 * per segment, in reverse, every pass of every step is recomputed with a record
 * of its input and its lambda, and the adjoint passes run in reverse from those
 * records (no root search in the adjoint).  With eslb_adjoint_tape_bytes of
 * workspace a segment is recomputed once, recording every step; with less, the
 * segment's step states are recomputed first and each step is run again,
 * recording, just before its adjoint passes.  The context's offsets are
 * unchanged on return.
 * Asynchronous. */
int eslb_adjoint(eslb_ctx* ctx, const double* f0_dev, int64_t nsteps, int64_t ckpt_every, double* fbar_dev,
                 void* work_dev, size_t work_bytes);
/* Device bytes of the checkpoints of (nsteps, ckpt_every): ceil(nsteps/ckpt_every)
 * states. */
int eslb_checkpoint_bytes(const eslb_ctx* ctx, int64_t nsteps, int64_t ckpt_every, size_t* bytes);
/* eslb_step(f_dev, nsteps) that also copies the state at steps 0, ckpt_every,
 * 2 ckpt_every, ... (storage layout, as it stands at that step) into ckpt_dev, a
 * caller-owned buffer of at least eslb_checkpoint_bytes bytes; a forward run that
 * keeps what eslb_adjoint_checkpointed needs.  Offsets advance as in eslb_step.
 * Asynchronous. */
int eslb_step_checkpointed(eslb_ctx* ctx, double* f_dev, int64_t nsteps, int64_t ckpt_every, double* ckpt_dev);
/* eslb_adjoint from the checkpoints of an eslb_step_checkpointed run instead of
 * its own forward sweep: the context's offsets must be those the run started
 * from (they are unchanged on return); ckpt_dev is read only; fbar_dev as in
 * eslb_adjoint.  work_dev: at least eslb_adjoint_workspace_bytes -
 * eslb_checkpoint_bytes bytes (taped with eslb_adjoint_tape_bytes -
 * eslb_checkpoint_bytes).  Same bits as eslb_adjoint.  Asynchronous. */
int eslb_adjoint_checkpointed(eslb_ctx* ctx, const double* ckpt_dev, int64_t nsteps, int64_t ckpt_every,
                              double* fbar_dev, void* work_dev, size_t work_bytes);

/* ---------------------------------------------------------------- batched ensembles
 * Many independent problems of one kind (same lattice, system, relax mode, scheme
 * and kappa; grid sizes, V, dx and system parameters may differ) advanced by one
 * stage kernel per pass over a device table of tiles of every active instance
 * (a persistent grid, or one block per tile: the launch configuration),
 * all instances in lockstep through the same composed-step schedule; the passes
 * of a few steps are captured in one hipGraph whose replays need no host work.
 * Not a method of the paper: an execution pattern for many problems at once; each
 * instance is computed exactly as eslb_step computes it. */
typedef struct eslb_batch eslb_batch;

/* probs: n problem statements (copied).  Every instance starts with offsets 0.
 * stream: the caller's stream (work is ordered after what is queued on it). */
int eslb_batch_create(const eslb_problem* probs, int32_t n, void* stream, eslb_batch** out);
void eslb_batch_destroy(eslb_batch* batch);
/* Advance instance i by nsteps[i] >= 0 composed steps, in place.  f_devs[i]: its
 * state (q*M planes of nx_i*ny_i, storage layout with the instance's offsets; may
 * be NULL when nsteps[i] == 0).  Synchronises with the batch's own stream before
 * returning (the caller's stream is made to wait for it as well).  Errors:
 * ESLB_ERR_INVALID_ARG (NULL argument, negative step count, a schedule of more
 * than 64 passes per step), ESLB_ERR_HIP. */
int eslb_batch_run(eslb_batch* batch, double* const* f_devs, const int64_t* nsteps);
/* Offsets of instance i (q entries, all equal: transport moves every velocity by
 * the same number of cells). */
int eslb_batch_get_offsets(const eslb_batch* batch, int32_t i, int64_t* offsets);
int eslb_batch_set_offsets(eslb_batch* batch, int32_t i, const int64_t* offsets);
/* Synchronise and return the sticky status of the whole batch. */
int eslb_batch_sync_status(eslb_batch* batch);
/* Launch configuration: tile block_x x block_y (64x4, 64x2, 128x2, 128x1, 256x1, 32x8),
 * blocks per compute unit of a persistent grid whose blocks take tiles from a
 * per-pass queue (0: one block per tile, dispatched by the hardware), composed
 * steps per captured graph.  Errors: ESLB_ERR_INVALID_ARG (NULL batch, a tile
 * shape not listed, blocks_per_cu < 0, steps_per_graph < 1). */
int eslb_batch_set_config(eslb_batch* batch, int32_t block_x, int32_t block_y, int32_t blocks_per_cu,
                          int32_t steps_per_graph);
int eslb_batch_get_config(const eslb_batch* batch, int32_t* cfg4);
/* Autotuner: for every supported configuration, builds the device tables and a
 * one-step graph once, then times max(replays, 3) graph replays with HIP events
 * (after one untimed replay) and keeps the configuration with the smallest
 * replay time; *best_ms (optional) gets that time.  The tuning set is a
 * systematic sample of at most 64 instances along the ensemble sorted by grid
 * size (its tile mix follows the ensemble's size distribution), run on scratch
 * copies that are allocated and freed here; the caller's states and offsets are
 * not modified.  Errors: ESLB_ERR_INVALID_ARG (NULL batch or states, replays < 1,
 * no non-NULL state), ESLB_ERR_HIP. */
int eslb_batch_autotune(eslb_batch* batch, double* const* f_devs, int32_t replays, double* best_ms);
const char* eslb_batch_last_error(const eslb_batch* batch);

const char* eslb_status_string(int code);
const char* eslb_last_error(const eslb_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ESLB_H */
