"""Batched ensemble (one stage kernel per pass over all instances, hipGraph-captured steps) against the plain
per-instance path and the oracle."""
import numpy as np
import pytest

from gpu_common import PARITY_RTOL, componentwise_error, oracle_system, to_gpu, to_host
from oracle.scheme import Relaxer, run
from oracle.systems import equilibrium
from paper_2403_13406_amd import workloads as W

pytestmark = pytest.mark.gpu


def ensemble(count, sizes, steps_range, seed=0):
    rng = np.random.default_rng(seed)
    ws = []
    for i in range(count):
        n = int(rng.choice(sizes))
        ny = int(rng.choice(sizes))
        ws.append(W.Workload("sw2d_t%d" % i, "D2Q4", "shallow_water", n, ny, 8.0, (9.81,),
                             int(rng.integers(*steps_range)), 1000 + i))
    return ws


def problem_kw(w):
    return dict(lattice=w.lattice, system=w.system, nx=w.nx, ny=w.ny, V=w.V, relax="entropic", param=w.param)


@pytest.mark.parametrize("config", [None, (64, 4, 2, 3), (256, 1, 8, 1), (32, 8, 4, 5), (64, 2, 0, 2)])
def test_batch_equals_per_instance_runs_bitwise(config):
    from paper_2403_13406_amd import Batch, Solver
    ws = ensemble(9, [13, 64, 70, 128], (1, 6))
    ws.append(W.Workload("sw2d_zero", "D2Q4", "shallow_water", 64, 64, 8.0, (9.81,), 0, 99))
    b = Batch([problem_kw(w) for w in ws])
    if config:
        b.set_config(*config)
    states, plain = [], []
    for w in ws:
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        f = s.init_equilibrium(to_gpu(w.initial_state()))
        states.append(f.clone())
        s.step(f, w.nsteps)
        s.sync()
        plain.append((to_host(f), s.offsets))
    b.run(states, [w.nsteps for w in ws])
    assert b.sync() == 0
    for i, w in enumerate(ws):
        assert b.offsets(i) == plain[i][1]
        assert np.array_equal(to_host(states[i]), plain[i][0]), i


def test_batch_against_oracle_and_second_run():
    from paper_2403_13406_amd import Batch, Solver
    ws = ensemble(4, [24, 40], (1, 4), seed=3)
    b = Batch([problem_kw(w) for w in ws])
    states, u0 = [], []
    for w in ws:
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        u = w.initial_state()
        u0.append(u)
        states.append(s.init_equilibrium(to_gpu(u)))
    steps = [w.nsteps for w in ws]
    b.run(states, steps)
    b.run(states, [2] * len(ws))          # continue from the offsets of the first run
    b.sync()
    for i, w in enumerate(ws):
        lat, sys = oracle_system(w.lattice, w.system, w.param)
        want = run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u0[i]), steps[i] + 2)
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        s.offsets = b.offsets(i)
        got = to_host(s.gather(states[i]))
        assert max(componentwise_error(got, want)) <= PARITY_RTOL


def test_autotune_leaves_states_untouched_and_picks_a_config():
    from paper_2403_13406_amd import Batch, Solver
    ws = ensemble(5, [64, 128], (2, 4), seed=4)
    b = Batch([problem_kw(w) for w in ws])
    states = []
    for w in ws:
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        states.append(s.init_equilibrium(to_gpu(w.initial_state())))
    before = [to_host(f) for f in states]
    cfg, ms = b.autotune(states)
    assert ms > 0 and cfg[0] * cfg[1] in (128, 256)
    for f, g in zip(states, before):
        assert np.array_equal(to_host(f), g)
    assert all(b.offsets(i) == [0] * 4 for i in range(len(ws)))


def test_batch_at_the_ensemble_sizes():
    """The first eight instances of the 512-instance ensemble (64^2 .. 1024^2 grids, their own initial
    data), one to three steps each so the active set shrinks during the run, autotuned as in the
    benchmark: bitwise equal to per-instance runs; the 1024^2 instance also sampled against the
    oracle on 81 x 81 periodic windows (one step moves a population by at most 36 cells)."""
    from paper_2403_13406_amd import Batch, Solver
    ws = W.sw2d_batch(8)
    steps = [3, 1, 2, 3, 1, 2, 3, 1]
    assert (ws[1].nx, ws[1].ny) == (1024, 1024)
    b = Batch([problem_kw(w) for w in ws])
    states, plain, u0 = [], [], []
    for w, n in zip(ws, steps):
        s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
        u = w.initial_state()
        u0.append(u)
        f = s.init_equilibrium(to_gpu(u))
        states.append(f.clone())
        s.step(f, n)
        assert s.sync() == 0
        plain.append((to_host(f), s.offsets))
    b.autotune(states)
    b.run(states, steps)
    assert b.sync() == 0
    for i in range(len(ws)):
        assert b.offsets(i) == plain[i][1]
        assert np.array_equal(to_host(states[i]), plain[i][0]), i
    w = ws[1]
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    s = Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax="entropic", param=w.param)
    s.offsets = b.offsets(1)
    g = to_host(s.gather(states[1]))
    R = 40
    for cy, cx in [(0, 1023), (600, 77)]:
        ys = (np.arange(-R, R + 1) + cy) % w.ny
        xs = (np.arange(-R, R + 1) + cx) % w.nx
        fw = run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u0[1][:, ys][:, :, xs]), 1)
        for m in range(fw.shape[1]):
            scale = np.max(np.abs(fw[:, m]))
            assert np.max(np.abs(g[:, m, cy, cx] - fw[:, m, R, R])) <= PARITY_RTOL * scale
