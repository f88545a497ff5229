"""Benchmark of the fourth-order entropy-stable LB time loop on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload euler2d|sw1d|burgers1d|batch|adjoint|aux|floor]

A "step" is one composed fourth-order step Phi(dt) (eq. splittingToUse): 18
passes "shift, entropic relax" over the whole grid.  The default workload is the
2D Euler D2Q4^4 grid of 4096^2 cells (FP64, entropy-limited omega); inputs are
seeded synthetic smooth fields resident in HBM before timing starts.

One JSON line:
  value        cells * K / timed seconds / 1e6 (MLUPS, whole job, one GPU)
  roofline     the stage kernel, timed with HIP events on the solver's stream
               around the timed steps (stage kernels only): algorithmic bytes per
               launch (2 q M 8 B per node) / average launch time vs 8 TB/s;
               traffic = rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (calibrated
               on a plain copy), from profiles/ when the kernel sources still match;
               floor (full run, 2D) = the same stage kernel with fixed omega
               (its loads and stores without the root search), same measure
  alu          (when profiles/ holds a VALU counter record of the same sources) the
               same launches against the FP64 vector peak and the VALU issue peak
  cpu_baseline the CPU oracle, single-threaded, on a bounded sample of the workload
  c1, c2       (default run) the 1D Burgers run (N = 1024, 17 steps to T = 0.2) and
               the 1D shallow-water run (N = 2^20, 4000 steps), whole runs timed
               with HIP events: MLUPS and ms per step
  batch        (default run) the 512-instance 2D shallow-water ensemble at its full
               step counts: one batch run (one stage kernel per pass over all
               instances, graph replays) vs the plain per-instance loop, same GPU
  adjoint      (default run) the 1024^2 Euler run of 2000 steps, checkpoints every
               50: forward vs forward+adjoint with the taped and the minimal
               workspace (peak device memory of each), and the gradient against
               central differences on the first 8 of the 32 seeded directions
  riemann      (default run) schemes (A), (B), (C) of Sec. 6.3 on the 2D Euler
               four-state Riemann problem to T = 0.25 at 1024^2 and 2048^2, wall
               seconds, with the paper's own (other GPU) times beside them
--workload batch / adjoint run only those two comparisons (the adjoint one with all 32
directions);
--workload aux times init, moments, gather and diagnostics at the 4096^2 Euler size;
--workload floor times only the fixed-omega stage pass of the roofline's floor.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak per 4th-order step; batched & adjoint vs plain same GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (FMA counted as two)
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9 / 1e12   # lane-slots/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz


def make_workload(name, size):
    from paper_2403_13406_amd import workloads as W
    if name == "euler2d":
        return W.euler2d(size or 4096)
    if name == "sw1d":
        return W.sw1d(size or (1 << 20))
    if name == "burgers1d":
        return W.burgers1d(size or 1024)
    raise SystemExit("unknown workload %s" % name)


def counter_record(kind, tag):
    """A committed rocprofv3 counter record (profiles/<kind>_<tag>.json) if the kernels still match it."""
    from paper_2403_13406_amd.profiling import source_hash
    path = os.path.join(ROOT, "profiles", "%s_%s.json" % (kind, tag))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec if rec.get("source_hash") == source_hash() else None


def cpu_baseline(w, budget_s=15.0):
    """The oracle (as it stands) timed on a bounded sample: the same generator on a small grid."""
    from threadpoolctl import threadpool_limits

    from oracle.lattice import Lattice
    from oracle.scheme import Relaxer, composed_step
    from oracle.systems import Burgers, Euler, ShallowWater, equilibrium
    from paper_2403_13406_amd import workloads as W

    if w.system == "euler":
        sample = W.euler2d(64, nsteps=1)
        lat, sys_ = Lattice("D2Q4"), Euler(w.param[0], 2)
    elif w.system == "shallow_water" and w.lattice == "D1Q2":
        sample = W.sw1d(4096, nsteps=1)
        lat, sys_ = Lattice("D1Q2"), ShallowWater(w.param[0], 1)
    elif w.system == "shallow_water":
        sample = W.Workload("sw2d_sample", "D2Q4", "shallow_water", 64, 64, 8.0, (9.81,), 1, 1000)
        lat, sys_ = Lattice("D2Q4"), ShallowWater(w.param[0], 2)
    else:
        sample = W.burgers1d(w.nx)
        lat, sys_ = Lattice("D1Q2"), Burgers((1.0,))
    u = sample.initial_state()
    with threadpool_limits(limits=1):
        f = equilibrium(lat, sys_, sample.V, u)
        r = Relaxer(lat, sys_, sample.V, "entropic")
        steps = 0
        t0 = time.perf_counter()
        while True:
            f = composed_step(r, f)
            steps += 1
            el = time.perf_counter() - t0
            if el > budget_s or steps >= 200:
                break
    cells = sample.nx * sample.ny
    return {"value": round(cells * steps / el / 1e6, 5), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%s %dx%d, %d composed entropic steps in %.1f s, numpy single thread"
                      % (sample.name, sample.nx, sample.ny, steps, el)}


def timed_steps(s, f, steps, torch):
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(s.stream)
    s.step(f, steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1)


def fixed_omega_floor(torch, w, steps=2):
    """The same stage kernel with fixed omega, per-pass launches (no fusion): the entropic
    pass's loads and stores with almost none of its arithmetic, i.e. the floor that this
    access pattern meets on this memory system."""
    from paper_2403_13406_amd import Solver
    u0 = torch.from_numpy(w.initial_state()).cuda()
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="fixed", omega=2.0, param=w.param, fused=False)
    f = s.init_equilibrium(u0)
    del u0
    s.step(f, 1)
    s.sync()
    ms = timed_steps(s, f, steps, torch)
    status = s.sync()   # reported, not asserted: this side measurement must not cost the bench line
    us = ms * 1e3 / (steps * 18)
    gbs = 2 * s.q * s.M * 8 * w.cells / (us * 1e-6) / 1e9
    del f
    s.close()
    return {"kernel": "the same stage kernel with fixed omega (no root search), per-pass launches",
            "us_per_launch": round(us, 2), "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "status": status}


def bench_single(args, torch):
    from paper_2403_13406_amd import Solver
    w = make_workload(args.workload, args.size)
    u0 = torch.from_numpy(w.initial_state()).cuda()
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax=w.relax, param=w.param)
    f = s.init_equilibrium(u0)
    del u0
    s.step(f, args.warmup)
    s.sync()
    ms = timed_steps(s, f, args.steps, torch)
    status = s.sync()
    if args.calibrate_copy_mib:
        # a plain device-to-device copy of known size, for the counter calibration
        n = args.calibrate_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    passes = 18
    avg_launch_s = ms / 1e3 / (args.steps * passes)
    bytes_per_launch = 2 * s.q * s.M * 8 * w.cells
    achieved = bytes_per_launch / avg_launch_s / 1e9
    tag = "%s_%dx%d" % (w.name, w.nx, w.ny)
    traffic = counter_record("traffic", tag)
    valu = counter_record("valu", tag)
    # the headline roofline: algorithmic bytes (2 q M 8 B per node, read and write of
    # every population once) over the stage kernel's average launch time, against HBM
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic["bytes_per_launch"]) if traffic else None,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    if traffic:
        roofline["traffic_over_algorithmic"] = round(traffic["bytes_per_launch"] / bytes_per_launch, 4)
    alu = None
    if valu:
        # secondary views of the same launches.  FP64 FLOPs per node (ADD + MUL + 2 FMA +
        # TRANS lane instructions) against the 78.6 TFLOP/s vector peak, and VALU issue
        # slots (every VALU instruction takes a SIMD's 16 lanes four cycles per wave, an
        # FP64 transcendental four times that) against the issue peak at 2.4 GHz and at
        # the clock the counters measured (GRBM_GUI_ACTIVE over the kernel time)
        tflops = valu["fp64_flop_per_node"] * w.cells / avg_launch_s / 1e12
        li = valu["lane_instructions_per_node"]
        slots = li["SQ_INSTS_VALU"] + 3.0 * li["SQ_INSTS_VALU_TRANS_F64"]
        issue = slots * w.cells / avg_launch_s / 1e12
        alu = {"fp64": {"achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "flop_per_node": valu["fp64_flop_per_node"]},
               "valu_issue": {"achieved": round(issue, 2), "peak": VALU_ISSUE_PEAK, "unit": "T lane-slots/s",
                              "frac": round(issue / VALU_ISSUE_PEAK, 4), "slots_per_node": slots}}
        clk = valu.get("clock_ghz")
        if clk:
            peak_clk = VALU_ISSUE_PEAK * clk / 2.4
            alu["valu_issue"].update({"clock_ghz_measured": clk, "peak_at_measured_clock": round(peak_clk, 2),
                                      "frac_at_measured_clock": round(issue / peak_clk, 4)})
    rec = {
        "metric": METRIC,
        "value": round(w.cells * args.steps / (ms / 1e3) / 1e6, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": tag, "lattice": w.lattice, "system": w.system, "nx": w.nx, "ny": w.ny,
                   "V": w.V, "relax": w.relax, "steps_in_workload": w.nsteps, "passes_per_step": passes},
        "roofline": roofline,
        "stage_kernel_avg_us": round(avg_launch_s * 1e6, 2),
        "status": status,
    }
    if alu:
        rec["alu"] = alu
    del f
    if not args.no_extras and w.lattice == "D2Q4":
        try:
            roofline["floor"] = fixed_omega_floor(torch, w)
        except Exception as e:  # noqa: BLE001  (a side measurement; the line stands without it)
            roofline["floor"] = {"error": "%s: %s" % (type(e).__name__, e)}
    return rec, w


def progress(msg):
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def batch_compare(torch, count, steps_scale, tune=True, seed_base=0):
    """Batched ensemble (one stage kernel per pass over all instances) vs the plain per-instance loop, same GPU."""

    from paper_2403_13406_amd import Batch, Solver
    from paper_2403_13406_amd import workloads as W
    ws = [W.sw2d_instance(i) for i in range(seed_base, seed_base + count)]
    steps = [max(1, int(round(w.nsteps * steps_scale))) for w in ws]
    b = Batch([dict(lattice=w.lattice, system=w.system, nx=w.nx, ny=w.ny, V=w.V, relax="entropic",
                    param=w.param) for w in ws])
    solvers, f_batch, f_plain = [], [], []
    for i, w in enumerate(ws):
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        f = s.init_equilibrium(torch.from_numpy(w.initial_state()).cuda())
        solvers.append(s)
        f_batch.append(f)
        f_plain.append(f.clone())
        if (i + 1) % 64 == 0:
            progress("batch: %d/%d instances initialised" % (i + 1, count))
    cfg = None
    if tune:
        cfg, _ = b.autotune(f_batch)
        progress("batch: autotuned config %s" % cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = list(steps)
    while max(left) > 0:     # chunks of at most 100 steps; the batch keeps every instance's offsets
        chunk = [min(100, n) for n in left]
        b.run(f_batch, chunk)
        left = [n - c for n, c in zip(left, chunk)]
        progress("batch: ensemble %d steps left at most (%.1f s)" % (max(left), time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    progress("batch: ensemble run %.2f s" % t_batch)
    t0 = time.perf_counter()
    for i, (s, f, n) in enumerate(zip(solvers, f_plain, steps)):
        s.step(f, n)
        if (i + 1) % 16 == 0:
            torch.cuda.synchronize()
            progress("batch: per-instance %d/%d (%.1f s)" % (i + 1, count, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(bool(torch.equal(a, c)) for a, c in zip(f_batch, f_plain))
    cell_steps = sum(w.cells * n for w, n in zip(ws, steps))
    return {"instances": count, "cells": sum(w.cells for w in ws), "cell_steps": cell_steps,
            "steps_scale": steps_scale, "batch_mlups": round(cell_steps / t_batch / 1e6, 2),
            "per_instance_mlups": round(cell_steps / t_plain / 1e6, 2),
            "speedup_vs_per_instance": round(t_plain / t_batch, 3), "bitwise_equal_to_per_instance": same,
            "autotuned_config": cfg, "batch_s": round(t_batch, 3), "per_instance_s": round(t_plain, 3),
            "ensemble_state_GiB": round(sum(f.numel() for f in f_batch) * 8 / 2 ** 30, 3)}


def adjoint_compare(torch, n, nsteps, ckpt, fd_dirs=0, minimal=True):
    """Forward vs forward + hand-written adjoint (checkpointing) for L = 1/2 |U(T) - U_target|^2.

    Both workspaces of the backward sweep are timed: "taped" (each segment recomputed once, its
    relaxation inputs kept) when it fits in half of the free device memory, and "minimal" (each
    segment recomputed twice, one state per step of a segment).  fd_dirs > 0 checks the gradient
    against central differences on the first fd_dirs of the seeded directions (seed 2)."""
    import numpy as np

    from paper_2403_13406_amd import Solver
    from paper_2403_13406_amd import workloads as W
    from paper_2403_13406_amd.autograd import time_loop
    w = W.euler2d_adjoint(n, nsteps=nsteps)
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
    u0 = torch.from_numpy(W.euler2d(n, seed=0, amp=0.005).initial_state()).cuda()
    ut = torch.from_numpy(W.euler2d(n, seed=1, amp=0.005).initial_state()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        uT = time_loop(u0, s, nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del uT
    progress("adjoint: forward %d steps %.2f s" % (nsteps, t_fwd))

    def fwd_adj(tape):
        x = u0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        L = 0.5 * torch.sum((time_loop(x, s, nsteps, ckpt, tape=tape) - ut) ** 2)
        L.backward()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        peak = torch.cuda.max_memory_allocated() - base
        progress("adjoint: forward + adjoint (%s) %.2f s, peak %.2f GiB above the inputs"
                 % ("taped" if tape else "minimal", sec, peak / 2 ** 30))
        return x.grad, sec, peak

    rec = {"grid": "%dx%d" % (n, n), "steps": nsteps, "ckpt_every": ckpt, "forward_s": round(t_fwd, 3),
           "state_GiB": round(s.q * s.M * n * n * 8 / 2 ** 30, 4)}
    nt = s.adjoint_tape_bytes(nsteps, ckpt)
    modes = []
    if nt <= torch.cuda.mem_get_info()[0] // 2:
        modes.append(("taped", True, nt))
    if minimal or not modes:
        modes.append(("minimal", False, s.adjoint_workspace_bytes(nsteps, ckpt)))
    g = None
    for i, (name, tape, ws) in enumerate(modes):
        if i == 0:
            fwd_adj(tape)     # the first call also allocates the workspace
        grad, sec, peak = fwd_adj(tape)
        g = grad if g is None else g
        rec[name] = {"forward_plus_adjoint_s": round(sec, 3), "ratio_to_forward": round(sec / t_fwd, 3),
                     "workspace_GiB": round(ws / 2 ** 30, 3), "peak_device_GiB": round(peak / 2 ** 30, 3)}
        torch.cuda.empty_cache()
    head = rec[modes[0][0]]
    rec["forward_plus_adjoint_s"] = head["forward_plus_adjoint_s"]
    rec["ratio_to_forward"] = head["ratio_to_forward"]
    rec["headline_workspace"] = modes[0][0]
    if fd_dirs:
        rng = np.random.default_rng(w.extra["fd_seed"])
        gnorm = float(torch.linalg.vector_norm(g))
        rel, proj = [], []
        for _ in range(fd_dirs):
            dl = torch.from_numpy(rng.standard_normal(tuple(u0.shape))).cuda()
            e = 1e-6
            with torch.no_grad():
                Lp = float(0.5 * torch.sum((time_loop(u0 + e * dl, s, nsteps) - ut) ** 2))
                Lm = float(0.5 * torch.sum((time_loop(u0 - e * dl, s, nsteps) - ut) ** 2))
            fd = (Lp - Lm) / (2 * e)
            ad = float(torch.sum(g * dl))
            rel.append(abs(fd - ad) / abs(fd))
            # |g.d| / (|g| |d|): how much of the gradient the direction sees
            proj.append(abs(ad) / (gnorm * float(torch.linalg.vector_norm(dl))))
            progress("adjoint: FD direction %d rel diff %.3e (|g.d|/|g||d| = %.2e)" % (len(rel), rel[-1], proj[-1]))
        rec["fd_directions"] = "the first %d of the %d seeded directions (seed %d), eps 1e-6" % (
            fd_dirs, w.extra["fd_dirs"], w.extra["fd_seed"])
        rec["fd_max_rel_diff"] = max(rel)
        rec["fd_median_rel_diff"] = float(np.median(rel))
        rec["fd_worst_direction_projection"] = proj[int(np.argmax(rel))]
        rec["fd_median_projection"] = float(np.median(proj))
    return rec


def single_run(torch, w, reps, warm_steps):
    """A whole run of a single-instance workload (w.nsteps composed steps from equilibrium), timed with
    HIP events on the solver's stream; the median over reps runs, each from a fresh initial state."""
    from paper_2403_13406_amd import Solver
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax=w.relax, param=w.param)
    u0 = torch.from_numpy(w.initial_state()).cuda()
    f = s.init_equilibrium(u0)
    s.step(f, warm_steps)
    s.sync()
    times = []
    for _ in range(reps):
        s.init_equilibrium(u0, f)      # offsets back to 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.step(f, w.nsteps)
        b.record(s.stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    assert s.sync() == 0
    d = s.diagnostics(f)
    times.sort()
    t = times[len(times) // 2]
    return {"workload": "%s_%d" % (w.name, w.nx), "cells": w.cells, "steps": w.nsteps, "runs": reps,
            "run_s": round(t, 6), "ms_per_step": round(t / w.nsteps * 1e3, 5),
            "mlups": round(w.cells * w.nsteps / t / 1e6, 2), "finite": d["n_nan"] == 0,
            "fallbacks": d["n_fallback"]}


# wall times of the three schemes of Sec. 6.3 on the paper's GPU (other hardware:
# context, not a target), seconds to T = 0.25
RIEMANN_PAPER_S = {1024: {"A": 7.213, "B": 6.072, "C": 9.470}, 2048: {"A": 59.697, "B": 53.270, "C": 64.529}}


def aux_kernels(torch, reps=20):
    """The kernels around the stage passes at the 4096^2 Euler size: eslb_init_equilibrium (a1),
    eslb_moments and eslb_gather (a3 observation, a2 layout), eslb_diagnostics (a7); HIP events on the
    solver stream, algorithmic bytes per call over the mean time."""
    from paper_2403_13406_amd import Solver
    w = make_workload("euler2d", 0)
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax=w.relax, param=w.param)
    u0 = torch.from_numpy(w.initial_state()).cuda()
    f = s.init_equilibrium(u0)
    s.step(f, 1)
    s.sync()
    q, M, cells = s.q, s.M, w.cells
    u = torch.empty_like(u0)
    g = torch.empty_like(f)

    def timed(fn):
        fn()
        s.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        for _ in range(reps):
            fn()
        b.record(s.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e3  # us per call

    out = {}
    for name, fn, nbytes in (
            ("moments", lambda: s.moments(f, u), (q * M + M) * 8 * cells),
            ("gather", lambda: s.gather(f, g), 2 * q * M * 8 * cells),
            ("init_equilibrium", lambda: s.init_equilibrium(u0, g), (M + q * M) * 8 * cells)):
        off = s.offsets
        us = timed(fn)
        s.offsets = off        # eslb_init_equilibrium starts a new state at offsets 0
        out[name] = {"us": round(us, 2), "GB/s": round(nbytes / us / 1e3, 1),
                     "frac_hbm": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 3)}
    t0 = time.perf_counter()
    for _ in range(reps):
        s.diagnostics(f)       # synchronous: includes the two read-backs
    out["diagnostics"] = {"us_synchronous": round((time.perf_counter() - t0) / reps * 1e6, 1),
                          "bytes_read": q * M * 8 * cells}
    return {"workload": "euler2d_%dx%d" % (w.nx, w.ny), "kernels": out}


def riemann_compare(torch, sizes=(1024, 2048)):
    """Sec. 6.3 timing: schemes (A), (B), (C) on the 2D Euler Riemann problem to T = 0.25."""
    from paper_2403_13406_amd import Solver
    from paper_2403_13406_amd import workloads as W
    out = {}
    for n in sizes:
        w = W.riemann2d(n)
        u0 = torch.from_numpy(w.initial_state()).cuda()
        row = {}
        for name, opts in W.RIEMANN_SCHEMES.items():
            s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, param=w.param, **opts)
            f = s.init_equilibrium(u0)
            steps = s.steps_for_time(w.extra["T"])
            s.sync()
            t0 = time.perf_counter()
            s.step(f, steps)
            s.sync()
            sec = time.perf_counter() - t0
            d = s.diagnostics(f)
            row[name] = {"steps": steps, "seconds": round(sec, 4), "finite": d["n_nan"] == 0,
                         "paper_seconds": RIEMANN_PAPER_S.get(n, {}).get(name)}
            del f
            progress("riemann %d^2: scheme %s, %d steps, %.3f s" % (n, name, steps, sec))
        out["%dx%d" % (n, n)] = row
        del u0
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="euler2d")
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reduced batch/adjoint comparisons and the Riemann-problem scheme timings")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0)
    ap.add_argument("--batch-steps-scale", type=float, default=1.0)
    ap.add_argument("--fd-dirs", type=int, default=None,
                    help="finite-difference directions of the adjoint check (default: 8 in the default run, 32 with --workload adjoint)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload == "batch":
        r = batch_compare(torch, 512, args.batch_steps_scale)
        rec = {"metric": METRIC, "value": r["batch_mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": None,
               "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic",
               "config": {"workload": "sw2d_batch_512", "lattice": "D2Q4", "system": "shallow_water"},
               "batch": r}
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "aux":
        r = aux_kernels(torch)
        print(json.dumps({"metric": "time and GB/s of the kernels around the stage passes", "n_gpus": 1,
                          "dtype": "f64", "data": "synthetic", "config": {"workload": r["workload"]},
                          "aux": r["kernels"]}), flush=True)
        return
    if args.workload == "floor":
        # the fixed-omega form of the 4096^2 Euler stage pass alone (the `floor` of the
        # default run's roofline), for a kernel trace of that measurement
        w = make_workload("euler2d", args.size)
        r = fixed_omega_floor(torch, w, steps=max(1, min(args.steps, 20)))
        print(json.dumps({"metric": "stage pass time, fixed omega", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "%s_%dx%d" % (w.name, w.nx, w.ny), "relax": "fixed"},
                          "floor": r}), flush=True)
        return
    if args.workload == "adjoint":
        r = adjoint_compare(torch, 1024, 2000, 50, 32 if args.fd_dirs is None else args.fd_dirs)
        rec = {"metric": METRIC, "value": round(1024 * 1024 * 2000 / r["forward_plus_adjoint_s"] / 1e6, 3),
               "unit": "MLUPS (forward+adjoint)", "n_gpus": 1, "steps": 2000, "warmup": 0, "ms_per_step": None,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", "config": {"workload": "euler2d_adjoint_1024x1024"}, "adjoint": r}
        print(json.dumps(rec), flush=True)
        return

    rec, w = bench_single(args, torch)

    def extra(key, fn):
        # a comparison that fails is recorded as such; it must not cost the headline line
        try:
            rec[key] = fn()
        except Exception as e:  # noqa: BLE001
            rec[key] = {"error": "%s: %s" % (type(e).__name__, e)}
        progress("%s: %s" % (key, rec[key]))
        torch.cuda.empty_cache()

    if not args.no_extras and args.workload == "euler2d":
        from paper_2403_13406_amd import workloads as W
        torch.cuda.empty_cache()
        extra("c1", lambda: single_run(torch, W.burgers1d(), reps=21, warm_steps=17))
        extra("c2", lambda: single_run(torch, W.sw1d(), reps=1, warm_steps=20))
        extra("batch", lambda: batch_compare(torch, 512, 1.0))
        extra("adjoint", lambda: adjoint_compare(torch, 1024, 2000, 50, 8 if args.fd_dirs is None else args.fd_dirs))
        extra("riemann", lambda: riemann_compare(torch))
    if not args.no_cpu_baseline:
        extra("cpu_baseline", lambda: cpu_baseline(w))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
