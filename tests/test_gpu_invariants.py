"""Per-step invariants of whole entropic runs on the GPU (Sec. 4), at full size.

The 1D Burgers run (N = 1024, V = 2, 17 composed steps to T = 0.2) and the 1D shallow-water run
(N = 2^20, g = 9.81, V = 4.5, all 4000 composed steps), advanced one step at a time, with the
library's deterministic diagnostics after every step:
  * sum_x u conserved: every stage moves populations (transport) or keeps the moments of a node
    (relaxation), so each step changes the sums by rounding only;
  * sum_x Sigma(f) conserved: with no omega = 1 fallback, each node's relaxation keeps its
    kinetic entropy (the root of F(-lambda) = F(1)) and the shifts permute nodes;
  * sum_x S(u_n) <= sum_x S(u_0): S(u) = Sigma(f^eq(u)) is the minimum of Sigma over
    populations with moments u, and the run starts at equilibrium;
  * no NaN, no node outside the convexity domain, no inadmissible state, no fallback.
Rounding bounds: a relaxation rounds each population once (relative 2^-53), the transport is
exact, so a step moves sum_x u_m by at most a few units of 2^-53 sum_x sum_k |f_{k,m}|; the
per-step bound below is 1e-14 of that scale, and the whole-run drift bound 1e-12.
"""
import pytest

from gpu_common import to_gpu
from paper_2403_13406_amd import workloads as W

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-14
RUN_TOL = 1e-12


@pytest.mark.parametrize("make", [W.burgers1d, W.sw1d], ids=["burgers1d_1024_17", "sw1d_2^20_4000"])
def test_whole_run_invariants(make):
    from paper_2403_13406_amd import Solver
    w = make()
    u0 = w.initial_state()
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
    f = s.init_equilibrium(to_gpu(u0))
    if w.name == "burgers1d":
        assert s.steps_for_time(0.2) == w.nsteps
    g0 = s.diagnostics(f)
    assert g0["n_outside"] == 0 and g0["n_nan"] == 0
    # the sums are rounded at the size of the populations: sum_x sum_k |f_{k,m}| (a moment may
    # vanish, as the shallow-water momentum does at t = 0, while its populations do not)
    scale_m = [1.5 * float(v) for v in f.abs().sum(dim=(0, 2, 3)).cpu()]
    scale_s = abs(g0["micro_entropy"])
    prev = g0
    worst_step = worst_run = worst_dS = 0.0
    for i in range(1, w.nsteps + 1):
        s.step(f, 1)
        g = s.diagnostics(f)
        assert g["n_nan"] == 0 and g["n_inadmissible"] == 0 and g["n_outside"] == 0, (i, g)
        assert g["n_fallback"] == 0, (i, g["n_fallback"])
        for m in range(len(scale_m)):
            ds = abs(g["mass"][m] - prev["mass"][m]) / scale_m[m]
            dr = abs(g["mass"][m] - g0["mass"][m]) / scale_m[m]
            worst_step, worst_run = max(worst_step, ds), max(worst_run, dr)
            assert ds <= STEP_TOL and dr <= RUN_TOL, (i, m, ds, dr)
        dS = abs(g["micro_entropy"] - prev["micro_entropy"]) / scale_s
        worst_dS = max(worst_dS, dS)
        assert dS <= STEP_TOL, (i, dS)
        assert abs(g["micro_entropy"] - g0["micro_entropy"]) <= RUN_TOL * scale_s, i
        assert g["macro_entropy"] <= g0["micro_entropy"] + STEP_TOL * scale_s, (i, g["macro_entropy"])
        prev = g
    assert s.sync() == 0
    print("%s: %d steps, max per-step mass change %.2e, max drift %.2e, max per-step entropy change %.2e "
          "(relative), macro entropy %.15e <= %.15e" % (w.name, w.nsteps, worst_step, worst_run, worst_dS,
                                                       g["macro_entropy"], g0["micro_entropy"]), flush=True)
