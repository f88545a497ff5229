"""Fused D1Q2 step (one kernel per composed step, all passes through LDS) against the
per-pass path, bit for bit, and against the oracle at sizes that span several blocks
with a ragged last block."""
import numpy as np
import pytest

from gpu_common import PARITY_RTOL, componentwise_error, oracle_system, to_gpu, to_host
from oracle.scheme import Relaxer, run
from oracle.systems import equilibrium
from paper_2403_13406_amd import workloads as W

pytestmark = pytest.mark.gpu

# owned cells per block: 32 KiB of LDS per window minus the halo (36 cells for Scheme I)
L_SW, L_SCALAR = 1024 - 72, 2048 - 72


def start_state(system, n, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(n) / n
    if system == "shallow_water":
        h = 1.0 + 0.1 * np.sin(2 * np.pi * x) + 0.02 * rng.standard_normal(n) * 0.01
        return np.stack([h, 0.05 * np.cos(2 * np.pi * x)])[:, None, :]
    return (0.5 + 0.25 * np.sin(2 * np.pi * x) + 0.01 * np.sin(6 * np.pi * x + rng.uniform()))[None, None, :]


# states above 64 KiB (smaller ones run in one workgroup), several blocks, ragged last block
CASES = [("shallow_water", (9.81,), 4.5, 3 * L_SW + 123), ("burgers", (1.0,), 2.0, 3 * L_SCALAR + 5),
         ("advection", (0.7,), 1.0, 3 * L_SCALAR + 1), ("shallow_water", (9.81,), 4.5, 5000)]


@pytest.mark.parametrize("system,param,V,n", CASES)
@pytest.mark.parametrize("relax,scheme", [("entropic", 1), ("fixed", 1), ("fixed", 2), ("fixed", 3),
                                          ("entropic", 3)])
def test_fused_step_equals_per_pass_path(system, param, V, n, relax, scheme):
    import torch

    from paper_2403_13406_amd import Solver
    a = Solver("D1Q2", system, n, 1, V=V, relax=relax, param=param, scheme=scheme, fused=True)
    b = Solver("D1Q2", system, n, 1, V=V, relax=relax, param=param, scheme=scheme, fused=False)
    assert a.step_work is not None and b.step_work is None
    u = to_gpu(start_state(system, n, 40))
    fa, fb = a.init_equilibrium(u), b.init_equilibrium(u)
    for k in (1, 2, 3):    # odd counts end with the copy back from the workspace
        a.step(fa, k)
        b.step(fb, k)
        assert a.sync() == 0 and b.sync() == 0
        assert a.offsets == b.offsets
        assert torch.equal(fa, fb), (k, float((fa - fb).abs().max()))


@pytest.mark.parametrize("system,param,V,n", CASES[:2])
def test_fused_step_against_oracle(system, param, V, n):
    from paper_2403_13406_amd import Solver
    lat, sys = oracle_system("D1Q2", system, param)
    u = start_state(system, n, 41)
    s = Solver("D1Q2", system, n, 1, V=V, relax="entropic", param=param, fused=True)
    assert s.step_work is not None
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, 3)
    assert s.sync() == 0
    want = run(Relaxer(lat, sys, V, "entropic"), equilibrium(lat, sys, V, u), 3)
    assert max(componentwise_error(to_host(s.gather(f)), want)) <= PARITY_RTOL


def test_fused_step_full_size_sw1d_sampled():
    """The 2^20-cell shallow-water workload: fused against per-pass after 2 steps (bitwise),
    and sampled cells against the oracle on a periodic window of 2 x 36 + 1 cells per step."""
    import torch

    from paper_2403_13406_amd import Solver
    w = W.sw1d()
    a = Solver(w.lattice, w.system, w.nx, 1, V=w.V, relax="entropic", param=w.param, fused=True)
    b = Solver(w.lattice, w.system, w.nx, 1, V=w.V, relax="entropic", param=w.param, fused=False)
    u = w.initial_state()
    fa, fb = a.init_equilibrium(to_gpu(u)), b.init_equilibrium(to_gpu(u))
    a.step(fa, 2)
    b.step(fb, 2)
    assert a.sync() == 0 and b.sync() == 0
    assert torch.equal(fa, fb)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    g = to_host(a.gather(fa))
    half = 2 * 36 + 8
    for x in np.random.default_rng(42).integers(0, w.nx, 6):
        idx = (np.arange(-half, half + 1) + x) % w.nx
        want = run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u[:, :, idx]), 2)
        got = g[:, :, :, idx]
        c = half
        scale = np.max(np.abs(want[:, :, :, c]))
        assert np.max(np.abs(got[:, :, :, c] - want[:, :, :, c])) <= PARITY_RTOL * scale


def test_fusion_policy():
    """"auto" takes the fused step for fixed omega and the entropic scalar systems, not for the
    entropic shallow-water pass; False never; True always (for grids above one workgroup)."""
    from paper_2403_13406_amd import Solver
    n = 6000
    assert Solver("D1Q2", "shallow_water", n, 1, V=4.5, relax="entropic", param=(9.81,)).step_work is None
    assert Solver("D1Q2", "shallow_water", n, 1, V=4.5, relax="fixed", param=(9.81,)).step_work is not None
    assert Solver("D1Q2", "burgers", n, 1, V=2.0, relax="entropic", param=(1.0,)).step_work is not None
    assert Solver("D1Q2", "burgers", n, 1, V=2.0, relax="fixed", param=(1.0,), fused=False).step_work is None
    assert Solver("D1Q2", "shallow_water", n, 1, V=4.5, relax="entropic", param=(9.81,),
                  fused=True).step_work is not None
    assert Solver("D1Q2", "burgers", 300, 1, V=2.0, param=(1.0,), fused=True).step_work is None  # one block
    assert Solver("D1Q2", "burgers", 1024, 1, V=2.0, param=(1.0,)).step_work is not None  # small: several CUs
    assert Solver("D2Q4", "burgers", 64, 64, V=2.0, param=(1.0, 0.5), fused=True).step_work is None


def test_step_workspace_errors():
    """A workspace smaller than one state and an unknown policy are rejected; detaching
    returns eslb_step to the per-pass path."""
    import ctypes

    import torch

    from paper_2403_13406_amd import _lib as L
    from paper_2403_13406_amd import Solver
    s = Solver("D1Q2", "burgers", 6000, 1, V=2.0, relax="fixed", param=(1.0,), fused=False)
    small = torch.empty(100, dtype=torch.uint8, device="cuda")
    assert s.lib.eslb_set_step_workspace(s.ctx, ctypes.c_void_p(small.data_ptr()), small.numel()) == L.ERR_INVALID_ARG
    assert s.lib.eslb_set_fusion(s.ctx, 7) == L.ERR_INVALID_ARG
    assert s.set_fused(True) is True and s.step_work is not None
    assert s.set_fused(False) is False and s.step_work is None


CASES_2D = [("euler", (1.4,), 3.2, 70, 61), ("shallow_water", (9.81,), 8.0, 83, 40), ("burgers", (1.0, 0.6), 2.0, 150, 33),
            ("advection", (0.3, 0.2), 1.0, 64, 64)]


def start_state_2d(system, nx, ny, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) / nx)[None, :]
    y = (np.arange(ny) / ny)[:, None]
    wave = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.01 * rng.standard_normal((ny, nx))
    if system == "euler":
        rho, vx, vy, p = 1 + 0.05 * wave, 0.05 * np.cos(2 * np.pi * y) + 0 * x, 0.03 * np.sin(2 * np.pi * x) + 0 * y, 1 + 0.02 * wave
        E = p / 0.4 + 0.5 * rho * (vx * vx + vy * vy)
        return np.stack([rho, rho * vx, rho * vy, E])
    if system == "shallow_water":
        h = 1 + 0.05 * wave
        return np.stack([h, 0.02 * h * np.cos(2 * np.pi * y) + 0 * x, 0.02 * h * np.sin(2 * np.pi * x) + 0 * y])
    return (0.3 + 0.05 * wave)[None]


@pytest.mark.parametrize("system,param,V,nx,ny", CASES_2D)
@pytest.mark.parametrize("scheme,omega", [(1, 2.0), (2, 2.0), (3, 2.0), (5, 1.93), (6, 2.0)])
def test_fused_2d_fixed_omega_equals_per_pass_path(system, param, V, nx, ny, scheme, omega):
    """D2Q4 fixed-omega segments through LDS (several tiles, ragged edges, every schedule):
    the same bits and offsets as the per-pass path after 1, 2 and 5 steps."""
    import torch

    from paper_2403_13406_amd import Solver
    a = Solver("D2Q4", system, nx, ny, V=V, relax="fixed", omega=omega, scheme=scheme, param=param)
    b = Solver("D2Q4", system, nx, ny, V=V, relax="fixed", omega=omega, scheme=scheme, param=param, fused=False)
    assert a.step_work is not None and b.step_work is None
    u = to_gpu(start_state_2d(system, nx, ny, 43))
    fa, fb = a.init_equilibrium(u), b.init_equilibrium(u)
    for k in (1, 2, 5):
        a.step(fa, k)
        b.step(fb, k)
        assert a.sync() == 0 and b.sync() == 0
        assert a.offsets == b.offsets
        assert torch.equal(fa, fb), (k, float((fa - fb).abs().max()))


def test_fused_2d_not_taken_for_entropic_omega():
    from paper_2403_13406_amd import Solver
    assert Solver("D2Q4", "euler", 128, 128, V=3.2, relax="entropic", param=(1.4,), fused=True).step_work is None
    assert Solver("D2Q4", "euler", 128, 128, V=3.2, relax="fixed", param=(1.4,)).step_work is not None


@pytest.mark.parametrize("lattice,system,param,V,nx,ny,kappa", [
    ("D2Q4", "burgers", (1.0, 0.6), 2.0, 150, 90, 2), ("D2Q4", "advection", (0.3, 0.2), 1.0, 160, 75, 3),
    ("D1Q2", "shallow_water", (9.81,), 4.5, 5000, 1, 3), ("D1Q2", "burgers", (1.0,), 2.0, 9000, 1, 2)])
def test_fused_larger_kappa(lattice, system, param, V, nx, ny, kappa):
    """Shifts of kappa cells per unit: longer halos (1D: 108 cells at kappa = 3), fewer passes per 2D segment
    (the scalar systems' 71-cell windows still fuse pairs of passes); fixed omega, the same bits and offsets
    as the per-pass path."""
    import torch

    from paper_2403_13406_amd import Solver
    a = Solver(lattice, system, nx, ny, V=V, kappa=kappa, relax="fixed", param=param, fused=True)
    b = Solver(lattice, system, nx, ny, V=V, kappa=kappa, relax="fixed", param=param, fused=False)
    assert a.step_work is not None
    u = start_state(system, nx, 44) if lattice == "D1Q2" else start_state_2d(system, nx, ny, 44)
    fa, fb = a.init_equilibrium(to_gpu(u)), b.init_equilibrium(to_gpu(u))
    a.step(fa, 3)
    b.step(fb, 3)
    assert a.sync() == 0 and b.sync() == 0
    assert a.offsets == b.offsets
    assert torch.equal(fa, fb)


@pytest.mark.parametrize("system,param,V,n,relax", [("burgers", (1.0,), 2.0, 1024, "entropic"),
                                                    ("shallow_water", (9.81,), 4.5, 1000, "entropic"),
                                                    ("advection", (0.7,), 1.0, 777, "fixed")])
def test_fused_small_states_equal_the_single_workgroup_run(system, param, V, n, relax):
    """States of at most 64 KiB: windows of one cell per thread over several blocks give the bits of
    the single-workgroup LDS run (and of the per-pass path); Scheme III too."""
    import torch

    from paper_2403_13406_amd import Solver
    for scheme in (1, 3):
        a = Solver("D1Q2", system, n, 1, V=V, relax=relax, param=param, scheme=scheme)
        b = Solver("D1Q2", system, n, 1, V=V, relax=relax, param=param, scheme=scheme, fused=False)
        assert a.step_work is not None and b.step_work is None
        u = to_gpu(start_state(system, n, 45))
        fa, fb = a.init_equilibrium(u), b.init_equilibrium(u)
        for k in (1, 2, 17):
            a.step(fa, k)
            b.step(fb, k)
            assert a.sync() == 0 and b.sync() == 0
            assert a.offsets == b.offsets
            assert torch.equal(fa, fb), (scheme, k)
