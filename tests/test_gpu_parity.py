"""HIP path (libeslb through its C ABI) against the CPU oracle, on the same seeded inputs.

Bar: transport bit-exact; states within 1e-12 per conserved component
(max |df_{k,m}| / max |f_{k,m}|) after one pass, one step and ten steps.
"""
import numpy as np
import pytest

from gpu_common import (PARITY_RTOL, componentwise_error, off_equilibrium, oracle_system, shifted_logical,
                        to_gpu, to_host)
from oracle.diagnostics import diagnostics as oracle_diagnostics
from oracle.lattice import Lattice, transport
from oracle.relaxation import relax_entropic, relax_fixed
from oracle.scheme import Relaxer, run
from oracle.systems import equilibrium
from paper_2403_13406_amd import workloads as W

pytestmark = pytest.mark.gpu


def solver_for(w, relax="entropic", scheme=1, omega=2.0):
    from paper_2403_13406_amd import Solver
    return Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, relax=relax, omega=omega, scheme=scheme, param=w.param)


def small(name):
    """Reduced-size versions of the workloads with ragged tails (not multiples of the block shape)."""
    if name == "burgers1d":
        return W.burgers1d(1024)
    if name == "sw1d":
        return W.sw1d(3000, nsteps=10)
    if name == "euler2d":
        return W.euler2d(70, ny=37, nsteps=10)
    if name == "sw2d":
        return W.Workload("sw2d_small", "D2Q4", "shallow_water", 67, 45, 8.0, (9.81,), 10, 5)
    if name == "burgers2d":
        return W.Workload("burgers2d_small", "D2Q4", "burgers", 50, 31, 2.0, (1.0, 0.6), 10, 3)
    if name == "advection2d":
        return W.Workload("advection2d_small", "D2Q4", "advection", 40, 33, 1.0, (0.2, -0.15), 10, 4)
    raise ValueError(name)


def initial_u(w):
    if w.name.startswith("burgers2d") or w.name.startswith("advection2d"):
        # smooth enough that Burgers stays shock-free over 10 steps (t = 2.4 at 50 x 31, V = 2)
        rng = np.random.default_rng(w.seed)
        return (0.3 + W.spectral_field_2d(w.nx, w.ny, rng, 1, 0.03))[None]
    return w.initial_state()


# ------------------------------------------------------------------ transport

@pytest.mark.parametrize("lattice,nx,ny", [("D1Q2", 1000, 1), ("D2Q4", 70, 37), ("D2Q4", 13, 5), ("D1Q2", 1, 1)])
def test_transport_bit_exact(lattice, nx, ny):
    """eq. transportPhase: stored state + offsets read back through eslb_gather equals numpy.roll, bit for bit."""
    from paper_2403_13406_amd import Solver
    lat = Lattice(lattice)
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 2 ** 63, size=(lat.q, 1, ny, nx), dtype=np.uint64)
    bits &= ~np.uint64(0x7FF0000000000000) | np.uint64(0x3FF0000000000000)   # no inf/NaN patterns
    f = bits.view(np.float64).copy()
    f.ravel()[0] = -0.0
    f.ravel()[-1] = 5e-324          # subnormal
    s = Solver(lattice, "advection", nx, ny, V=1.0, relax="fixed", param=(0.1, 0.1))
    fg = to_gpu(f)
    for offs in ([0] * lat.q, [1] * lat.q, [-4, 2, 7, -9][:lat.q], [123456789, -77, 3, 2 ** 40 + 5][:lat.q]):
        s.offsets = offs
        g = to_host(s.gather(fg))
        want = shifted_logical(lat, f, offs)
        assert np.array_equal(g.view(np.uint64), want.view(np.uint64))
    # the step's shift bookkeeping: one composed step moves every velocity by 24 kappa cells
    s.offsets = [0] * lat.q
    s2 = Solver(lattice, "advection", nx, ny, V=1.0, relax="fixed", param=(0.1, 0.1), kappa=2)
    s2.step(s2.empty_state().zero_(), 1)
    assert s2.offsets == [48] * lat.q


# ------------------------------------------------------------------ one relaxation pass

@pytest.mark.parametrize("name", ["burgers1d", "sw1d", "euler2d", "sw2d", "burgers2d", "advection2d"])
@pytest.mark.parametrize("relax", ["fixed", "entropic"])
@pytest.mark.parametrize("shift", [1, -4])
def test_one_pass(name, relax, shift):
    """One stage T(shift) R: eq. transportPhase then eq. relaxationDiscretizationOmega / variableOmegaProblem."""
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = initial_u(w)
    f0 = off_equilibrium(lat, sys, w.V, u, shift=2)
    s = solver_for(w, relax)
    fg = to_gpu(f0)
    s.transport(shift)
    s.relax(fg)
    assert s.sync() == 0
    got = to_host(s.gather(fg))
    g = transport(lat, f0, shift)
    want = relax_fixed(lat, sys, w.V, g, 2.0) if relax == "fixed" else relax_entropic(lat, sys, w.V, g)
    err = componentwise_error(got, want)
    assert max(err) <= PARITY_RTOL, err


@pytest.mark.parametrize("system,rel", [("euler", 0.01), ("euler", 0.05), ("euler", 0.15), ("shallow_water", 0.05),
                                        ("shallow_water", 0.15), ("shallow_water", 0.3)])
def test_one_pass_far_from_equilibrium(system, rel):
    """Entropic relaxation of stage inputs far from equilibrium (relative offsets of f from f^eq up to rel):
    the population-state offsets reach |z| >= 2^-7, past the series range of the Bregman terms, and the
    predictor shortcut does not apply."""
    lat, sys = oracle_system("D2Q4", system, (1.4,) if system == "euler" else (9.81,))
    V = 3.2 if system == "euler" else 8.0
    nx, ny = 67, 29
    rng = np.random.default_rng(31)
    if system == "euler":
        u = W.euler2d(nx, ny=ny, amp=0.1).initial_state()
    else:
        u = np.stack([1.0 + 0.05 * rng.standard_normal((ny, nx)), 0.05 * rng.standard_normal((ny, nx)),
                      0.05 * rng.standard_normal((ny, nx))])
    feq = equilibrium(lat, sys, V, u)
    f0 = feq + rel * np.abs(feq) * rng.uniform(-1.0, 1.0, feq.shape)
    from paper_2403_13406_amd import Solver
    s = Solver("D2Q4", system, nx, ny, V=V, relax="entropic", param=(1.4,) if system == "euler" else (9.81,))
    fg = to_gpu(f0)
    s.relax(fg)
    s.sync()
    want = relax_entropic(lat, sys, V, f0)
    got = to_host(fg)
    err = componentwise_error(got, want)
    assert max(err) <= PARITY_RTOL, err


@pytest.mark.parametrize("system,param,V,rel", [("shallow_water", (9.81,), 4.5, 0.05), ("shallow_water", (9.81,), 4.5, 0.2),
                                                ("burgers", (1.0,), 2.0, 0.05), ("burgers", (1.0,), 2.0, 0.3)])
def test_one_pass_far_from_equilibrium_1d(system, param, V, rel):
    """D1Q2 entropic relaxation of stage inputs with relative offsets from f^eq up to rel."""
    lat, sys = oracle_system("D1Q2", system, param)
    n = 3001
    rng = np.random.default_rng(32)
    if system == "shallow_water":
        u = np.stack([1.0 + 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n)])[:, None, :]
    else:
        u = (0.4 + 0.1 * rng.standard_normal(n))[None, None, :]
    feq = equilibrium(lat, sys, V, u)
    f0 = feq + rel * np.abs(feq) * rng.uniform(-1.0, 1.0, feq.shape)
    from paper_2403_13406_amd import Solver
    s = Solver("D1Q2", system, n, 1, V=V, relax="entropic", param=param)
    fg = to_gpu(f0)
    s.relax(fg)
    s.sync()
    err = componentwise_error(to_host(fg), relax_entropic(lat, sys, V, f0))
    assert max(err) <= PARITY_RTOL, err


# ------------------------------------------------------------------ composed steps

@pytest.mark.parametrize("name,nsteps", [("burgers1d", 17), ("sw1d", 1), ("sw1d", 10), ("euler2d", 1), ("euler2d", 10),
                                         ("sw2d", 10), ("burgers2d", 10), ("advection2d", 3)])
def test_composed_steps_entropic(name, nsteps):
    """n steps of Phi (eq. splittingToUse) with the entropy-limited omega, from equilibrium data."""
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = initial_u(w)
    s = solver_for(w, "entropic")
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, nsteps)
    assert s.sync() == 0
    got = to_host(s.gather(f))
    want = run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u), nsteps)
    err = componentwise_error(got, want)
    assert max(err) <= PARITY_RTOL, err
    um = to_host(s.moments(f))
    assert np.max(np.abs(um - want.sum(0))) <= PARITY_RTOL * 4 * np.max(np.abs(want.sum(0)))


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_composed_steps_fixed_omega_and_projection_schemes(scheme):
    """omega = 2 (Sec. 2-3) and Schemes II, III of Sec. 6.1 on Burgers."""
    w = W.burgers1d(640)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = w.initial_state()
    s = solver_for(w, "fixed", scheme=scheme)
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, 4)
    s.sync()
    want = run(Relaxer(lat, sys, w.V, "fixed"), equilibrium(lat, sys, w.V, u), 4, scheme=scheme)
    assert max(componentwise_error(to_host(s.gather(f)), want)) <= PARITY_RTOL


def test_full_size_euler_step_sampled():
    """One composed step of the 4096^2 Euler workload in the benchmark's launch shape; sampled nodes
    are checked against the oracle run on a 73 x 73 periodic window around each (one step moves
    populations by at most 36 cells, so the window centre is exact)."""
    w = W.euler2d()
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = w.initial_state()
    s = solver_for(w, "entropic")
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, 1)
    assert s.sync() == 0
    g = s.gather(f)
    rng = np.random.default_rng(12)
    R = 36
    for _ in range(4):
        cy, cx = (int(v) for v in rng.integers(0, 4096, size=2))
        ys = (np.arange(cy - R, cy + R + 1)) % 4096
        xs = (np.arange(cx - R, cx + R + 1)) % 4096
        uw = u[:, ys][:, :, xs]
        fw = run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, uw), 1)
        want = fw[:, :, R, R]
        got = to_host(g[:, :, cy, cx])
        for m in range(4):
            scale = np.max(np.abs(fw[:, m]))      # max |f_{k,m}| over the window
            assert np.max(np.abs(got[:, m] - want[:, m])) <= PARITY_RTOL * scale


# ------------------------------------------------------------------ diagnostics and edge cases

@pytest.mark.parametrize("name", ["sw1d", "euler2d", "burgers1d"])
def test_diagnostics(name):
    """Conserved sums and entropies (Sec. 4) against the oracle's exactly rounded sums."""
    w = small(name)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = initial_u(w)
    s = solver_for(w, "entropic")
    s.set_stats(True)
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, 2)
    d = s.diagnostics(f)
    want = oracle_diagnostics(lat, sys, w.V, run(Relaxer(lat, sys, w.V, "entropic"), equilibrium(lat, sys, w.V, u), 2))
    for a, b in zip(d["mass"], want["mass"]):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b))
    assert abs(d["micro_entropy"] - want["micro_entropy"]) <= 1e-11 * abs(want["micro_entropy"])
    assert abs(d["macro_entropy"] - want["macro_entropy"]) <= 1e-11 * abs(want["macro_entropy"])
    assert d["n_fallback"] == 0 and d["n_outside"] == 0 and d["n_nan"] == 0
    assert 1.9 < d["omega_min"] <= d["omega_max"] < 2.1


def test_exact_translation_bit_exact():
    """a = V: R is the identity and u(t_n) is u0 moved by 24 n cells, bit for bit."""
    from paper_2403_13406_amd import Solver
    n = 96
    u0 = np.random.default_rng(13).standard_normal((1, 1, n))
    for relax in ("fixed", "entropic"):
        s = Solver("D1Q2", "advection", n, 1, V=1.0, relax=relax, param=(1.0,))
        with pytest.warns(RuntimeWarning):      # a = V sits on the sub-characteristic limit
            f = s.init_equilibrium(to_gpu(u0))
        s.step(f, 3)
        s.sync()
        assert np.array_equal(to_host(s.moments(f))[0, 0], np.roll(u0[0, 0], 72))


def test_fallback_and_errors():
    """Silent cases, read as: no entropic root => omega = 1 and a warning; bad input => error codes."""
    from paper_2403_13406_amd import EslbError, Solver
    s = Solver("D1Q2", "burgers", 8, 1, V=1.0, relax="entropic", param=(1.0,))
    lat, sys = oracle_system("D1Q2", "burgers", (1.0,))
    f = equilibrium(lat, sys, 1.0, np.full((1, 1, 8), 0.2))
    f[0, 0, 0, 3] -= 0.4
    f[1, 0, 0, 3] += 0.4
    fg = to_gpu(f)
    s.relax(fg)
    with pytest.warns(RuntimeWarning):
        assert s.sync() == 1
    got = to_host(fg)
    want = relax_entropic(lat, sys, 1.0, f)
    assert np.max(np.abs(got - want)) <= 1e-15
    with pytest.raises(EslbError):
        Solver("D1Q2", "euler", 8, 1, V=1.0, param=(1.4,))
    with pytest.raises(EslbError):
        Solver("D2Q4", "euler", 0, 8, V=1.0, param=(1.4,))
    sw = Solver("D1Q2", "shallow_water", 8, 1, V=4.0, param=(9.81,))
    u = np.ones((2, 1, 8))
    u[0, 0, 2] = -1.0
    with pytest.raises(EslbError):
        sw.init_equilibrium(to_gpu(u))


@pytest.mark.parametrize("lattice,system,nx,ny,V,param,scheme", [
    ("D1Q2", "burgers", 1024, 1, 2.0, (1.0,), 1),
    ("D1Q2", "shallow_water", 1000, 1, 4.5, (9.81,), 1),
    ("D2Q4", "burgers", 40, 31, 2.0, (1.0, 0.6), 1),
    ("D2Q4", "shallow_water", 24, 20, 8.0, (9.81,), 1),
    ("D2Q4", "euler", 16, 12, 3.2, (1.4,), 1),
    ("D1Q2", "burgers", 640, 1, 2.0, (1.0,), 3),
])
def test_whole_run_in_lds_equals_pass_by_pass(lattice, system, nx, ny, V, param, scheme):
    """States of at most 64 KiB run all passes in one workgroup's LDS; bits must equal the per-pass path."""
    from paper_2403_13406_amd import Solver
    lat, sys = oracle_system(lattice, system, param)
    rng = np.random.default_rng(14)
    if system == "burgers":
        u = 0.3 + 0.02 * rng.standard_normal((1, ny, nx))
    elif system == "shallow_water":
        h = 1.0 + 0.01 * rng.standard_normal((ny, nx))
        u = np.stack([h] + [0.01 * rng.standard_normal((ny, nx)) for _ in range(lat.d)])
    else:
        w = W.euler2d(nx, ny=ny)
        u = w.initial_state()
    runs = []
    for track in (False, True):        # stats tracking forces one launch per pass
        s = Solver(lattice, system, nx, ny, V=V, relax="entropic", scheme=scheme, param=param, fused=False)
        s.set_stats(track)
        f = s.init_equilibrium(to_gpu(u))
        s.transport(3)                 # start from unequal-to-zero offsets
        s.step(f, 3)
        s.sync()
        runs.append((to_host(f), s.offsets, to_host(s.gather(f))))
    assert runs[0][1] == runs[1][1]
    assert np.array_equal(runs[0][0], runs[1][0])
    want = run(Relaxer(lat, sys, V, "entropic"), transport(lat, equilibrium(lat, sys, V, u), 3), 3, scheme=scheme)
    assert max(componentwise_error(runs[0][2], want)) <= PARITY_RTOL


@pytest.mark.parametrize("scheme", [4, 5, 6])
@pytest.mark.parametrize("relax", ["fixed", "entropic"])
def test_comparison_schedules(scheme, relax):
    """Standard LB comparator (Sec. 3.1) and Schemes (A), (B) of Sec. 6.3, on 2D Euler and 1D Burgers."""
    from oracle.scheme import scheme_A_step, scheme_B_step, standard_lb_step
    step = {4: standard_lb_step, 5: scheme_A_step, 6: scheme_B_step}[scheme]
    for w in (W.euler2d(70, ny=37), W.burgers1d(3000)):
        lat, sys = oracle_system(w.lattice, w.system, w.param)
        u = w.initial_state()
        omega = 1.93 if (scheme == 5 and relax == "fixed") else 2.0
        s = solver_for(w, relax, scheme=scheme, omega=omega)
        f = s.init_equilibrium(to_gpu(u))
        s.step(f, 3)
        assert s.sync() == 0
        r = Relaxer(lat, sys, w.V, relax, omega)
        want = equilibrium(lat, sys, w.V, u)
        for _ in range(3):
            want = step(r, want)
        assert max(componentwise_error(to_host(s.gather(f)), want)) <= PARITY_RTOL
        net = {4: 24, 5: 1, 6: 4}[scheme]
        assert abs(s.dt() - net * w.dx / w.V) <= 1e-15 * s.dt()


def test_failure_injection_nan_inadmissible_subcharacteristic():
    """Forced from the host: a NaN population, an inadmissible cell met by a relaxation pass, and V
    below the sub-characteristic bound report their status codes (sticky until the counters reset)."""
    from paper_2403_13406_amd import EslbError, Solver
    from paper_2403_13406_amd import _lib as L
    lat, sys = oracle_system("D1Q2", "shallow_water", (9.81,))
    # NaN in one population: the pass flags it
    s = Solver("D1Q2", "shallow_water", 64, 1, V=4.5, relax="entropic", param=(9.81,))
    f = equilibrium(lat, sys, 4.5, np.stack([np.ones(64), np.zeros(64)])[:, None, :])
    f[0, 0, 0, 5] = np.nan
    fg = to_gpu(f)
    s.relax(fg)
    with pytest.raises(EslbError) as e:
        s.sync()
    assert e.value.code == L.ERR_NAN
    # a cell whose moments are inadmissible (h < 0) reaching a relaxation
    s2 = Solver("D1Q2", "shallow_water", 64, 1, V=4.5, relax="entropic", param=(9.81,))
    f = equilibrium(lat, sys, 4.5, np.stack([np.ones(64), np.zeros(64)])[:, None, :])
    f[:, 0, 0, 9] *= -1.0
    fg = to_gpu(f)
    s2.relax(fg)
    with pytest.raises(EslbError) as e:
        s2.sync()
    assert e.value.code == L.ERR_INADMISSIBLE
    s2.reset_counters()
    s2.relax(to_gpu(equilibrium(lat, sys, 4.5, np.stack([np.ones(64), np.zeros(64)])[:, None, :])))
    assert s2.sync() == 0    # the sticky status is cleared by the reset
    # V below |u| + sqrt(g h): the initialisation warns
    s3 = Solver("D1Q2", "shallow_water", 64, 1, V=2.0, relax="fixed", param=(9.81,))
    with pytest.warns(RuntimeWarning):
        s3.init_equilibrium(to_gpu(np.stack([np.ones(64), np.zeros(64)])[:, None, :]))
        assert s3.sync() == L.WARN_SUBCHARACTERISTIC
