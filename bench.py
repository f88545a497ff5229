"""Benchmark of the fourth-order entropy-stable LB time loop on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload euler2d|sw1d|burgers1d]

A "step" is one composed fourth-order step Phi(dt) (eq. splittingToUse): 18
passes "shift, entropic relax" over the whole grid.  The default workload is the
2D Euler D2Q4^4 grid of 4096^2 cells (FP64, entropy-limited omega); inputs are
seeded synthetic smooth fields resident in HBM before timing starts.

Prints one JSON line:
  value      = cells * K / timed seconds / 1e6 (MLUPS, whole job, one GPU)
  roofline   = the stage kernel: algorithmic bytes per launch (2 q M 8 B per cell)
               / its average launch duration (HIP events on the solver's stream over
               the timed region, which holds stage kernels only) vs 8 TB/s HBM
  cpu_baseline = the CPU oracle, single-threaded, on a bounded sample of the same
               workload (a smaller grid of the same generator), in MLUPS.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak per 4th-order step; batched & adjoint vs plain same GPU"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_13406_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name, size):
    from paper_2403_13406_amd import workloads as W
    if name == "euler2d":
        return W.euler2d(size or 4096)
    if name == "sw1d":
        return W.sw1d(size or (1 << 20))
    if name == "burgers1d":
        return W.burgers1d(size or 1024)
    raise SystemExit("unknown workload %s" % name)


def traffic_for(workload_tag):
    """HBM bytes per stage launch from committed rocprofv3 --pmc summaries, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload_tag)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(w, budget_s=15.0):
    """Time the oracle (as it stands) on a bounded sample: the same generator on a small grid."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.lattice import Lattice
    from oracle.scheme import Relaxer, composed_step
    from oracle.systems import Burgers, Euler, ShallowWater, equilibrium
    from paper_2403_13406_amd import workloads as W

    if w.system == "euler":
        sample = W.euler2d(64, nsteps=1)
        lat, sys_ = Lattice("D2Q4"), Euler(w.param[0], 2)
    elif w.system == "shallow_water":
        sample = W.sw1d(4096, nsteps=1)
        lat, sys_ = Lattice("D1Q2"), ShallowWater(w.param[0], 1)
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
            if el > budget_s or steps >= sample.nsteps * 50:
                break
    cells = sample.nx * sample.ny
    return {"value": cells * steps / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "%s %dx%d, %d composed entropic steps, %.1f s, numpy single thread"
                      % (sample.name, sample.nx, sample.ny, steps, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="euler2d")
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2403_13406_amd import Solver

    w = make_workload(args.workload, args.size)
    u0 = torch.from_numpy(w.initial_state()).cuda()
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax=w.relax, param=w.param)
    f = s.init_equilibrium(u0)
    del u0
    s.step(f, args.warmup)
    s.sync()
    stream = s.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    s.step(f, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    status = s.sync()
    cells = w.cells
    value = cells * args.steps / (ms / 1e3) / 1e6
    passes = 18
    avg_launch_s = ms / 1e3 / (args.steps * passes)
    bytes_per_launch = 2 * s.q * s.M * 8 * cells
    achieved = bytes_per_launch / avg_launch_s / 1e9
    tag = "%s_%dx%d" % (w.name, w.nx, w.ny)
    traffic = traffic_for(tag)
    rec = {
        "metric": METRIC,
        "value": round(value, 3),
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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "stage_kernel_avg_us": round(avg_launch_s * 1e6, 2),
        "status": status,
        "source_hash": source_hash(),
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
