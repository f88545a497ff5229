"""2D Euler Riemann problem with four constant states (Sec. 6.3 setting).

Schemes (A), (B) and (C) of Sec. 6.3 on discontinuous data: the GPU path
against the oracle element by element on a small grid, then a run to the
paper's final time that must stay finite and conservative.  The four states are
our own (see workloads.riemann2d); the domain is periodic.
"""
import numpy as np
import pytest

from gpu_common import PARITY_RTOL, componentwise_error, oracle_system, to_gpu, to_host
from oracle.scheme import Relaxer, composed_step, scheme_A_step, scheme_B_step
from oracle.systems import equilibrium
from paper_2403_13406_amd import workloads as W

pytestmark = pytest.mark.gpu


def oracle_step(name):
    return {"A": scheme_A_step, "B": scheme_B_step, "C": lambda r, f: composed_step(r, f, scheme=3)}[name]


def solver(w, name):
    from paper_2403_13406_amd import Solver
    return Solver(w.lattice, w.system, w.nx, w.ny, V=w.V, param=w.param, **W.RIEMANN_SCHEMES[name])


@pytest.mark.parametrize("name,steps", [("A", 12), ("B", 4), ("C", 2)])
def test_riemann_schemes_match_oracle(name, steps):
    w = W.riemann2d(48)
    lat, sys = oracle_system(w.lattice, w.system, w.param)
    u = w.initial_state()
    s = solver(w, name)
    f = s.init_equilibrium(to_gpu(u))
    s.step(f, steps)
    assert s.sync() == 0
    r = Relaxer(lat, sys, w.V, "fixed", W.RIEMANN_SCHEMES[name]["omega"])
    want = equilibrium(lat, sys, w.V, u)
    for _ in range(steps):
        want = oracle_step(name)(r, want)
    assert max(componentwise_error(to_host(s.gather(f)), want)) <= PARITY_RTOL


@pytest.mark.parametrize("name", ["A", "B", "C"])
def test_riemann_schemes_reach_final_time(name):
    """256^2 to T = 0.25: no NaN, conserved totals kept to rounding."""
    w = W.riemann2d(256)
    u = w.initial_state()
    s = solver(w, name)
    f = s.init_equilibrium(to_gpu(u))
    n = s.steps_for_time(w.extra["T"])
    assert n * s.dt() <= w.extra["T"] < (n + 1) * s.dt()
    s.step(f, n)
    d = s.diagnostics(f)
    assert d["n_nan"] == 0 and d["n_inadmissible"] == 0
    uT = to_host(s.moments(f))
    assert np.all(np.isfinite(uT))
    for m in range(4):
        assert abs(uT[m].sum() - u[m].sum()) <= 1e-12 * np.abs(u[m]).sum()
    assert uT[0].min() > 0.0
