"""Pins of the oracle adjoint: exact transpose in the linear case, finite differences otherwise.

The adjoint is not in the paper; what fixes it is the definition of the
derivative of the paper's scheme.
"""
import numpy as np
import pytest

from oracle.adjoint import adjoint_run, eq_jacobian_T, misfit_gradient, relax_adjoint
from oracle.lattice import Lattice, transport
from oracle.relaxation import relax_entropic, relax_fixed
from oracle.scheme import Relaxer, run
from oracle.systems import Advection, equilibrium
from test_oracle_pins import SYSTEMS, shape_of, smooth_state

D1 = Lattice("D1Q2")
D2 = Lattice("D2Q4")


@pytest.mark.parametrize("lat,a", [(D1, (0.3,)), (D2, (0.2, -0.1))])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_linear_adjoint_is_the_exact_transpose(lat, a, scheme):
    """Linear flux, fixed omega: Phi is a linear map, so <Phi^n v, w> = <v, Phi^{n,T} w> to rounding."""
    rng = np.random.default_rng(20)
    shp = (lat.q, 1, 1, 40) if lat.d == 1 else (lat.q, 1, 9, 11)
    v = rng.standard_normal(shp)
    w = rng.standard_normal(shp)
    r = Relaxer(lat, Advection(a), 1.0, "fixed")
    lhs = np.sum(run(r, v, 2, scheme=scheme) * w)
    rhs = np.sum(v * adjoint_run(r, v, 2, w, scheme=scheme))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_equilibrium_jacobian_transpose_by_finite_differences():
    rng = np.random.default_rng(21)
    lat, sys, V, u = smooth_state("euler2d", (4, 5), rng)
    u = u.reshape(4, -1)
    y = rng.standard_normal((4, 4, u.shape[1]))
    dl = rng.standard_normal(u.shape)
    e = 1e-6
    jv = (equilibrium(lat, sys, V, u + e * dl) - equilibrium(lat, sys, V, u - e * dl)) / (2 * e)
    assert abs(np.sum(jv * y) - np.sum(dl * eq_jacobian_T(lat, sys, V, u, y))) <= 1e-8 * np.sum(np.abs(jv * y))


@pytest.mark.parametrize("name", SYSTEMS)
@pytest.mark.parametrize("mode", ["fixed", "entropic"])
def test_stage_adjoint_against_central_differences(name, mode):
    """<(R(h + e v) - R(h - e v)) / 2e, w> = <v, R'(h)^T w>: the derivative of omega(h) included."""
    rng = np.random.default_rng(22)
    lat, sys, V, u = smooth_state(name, shape_of(name), rng)
    h = transport(lat, equilibrium(lat, sys, V, u), 2)
    v = rng.standard_normal(h.shape)
    w = rng.standard_normal(h.shape)
    e = 1e-6
    R = (lambda x: relax_fixed(lat, sys, V, x, 2.0)) if mode == "fixed" else (lambda x: relax_entropic(lat, sys, V, x))
    jv = (R(h + e * v) - R(h - e * v)) / (2 * e)
    lhs = np.sum(jv * w)
    rhs = np.sum(v * relax_adjoint(lat, sys, V, h, w, mode))
    assert abs(lhs - rhs) <= 2e-8 * np.sum(np.abs(jv * w))


@pytest.mark.parametrize("name", ["euler2d", "sw1d"])
def test_misfit_gradient_against_central_differences(name):
    """dL/du0 of L = 1/2 |U(T) - U_target|^2 through two entropic composed steps."""
    rng = np.random.default_rng(23)
    lat, sys, V, u = smooth_state(name, shape_of(name), rng)
    ut = u * (1 + 0.01 * rng.standard_normal(u.shape))
    r = Relaxer(lat, sys, V, "entropic")
    L, g = misfit_gradient(r, u, ut, 2)

    def loss(x):
        return 0.5 * np.sum((run(r, equilibrium(lat, sys, V, x), 2).sum(0) - ut) ** 2)

    assert abs(L - loss(u)) <= 1e-14 * L
    for _ in range(3):
        dl = rng.standard_normal(u.shape)
        e = 1e-6
        fd = (loss(u + e * dl) - loss(u - e * dl)) / (2 * e)
        assert abs(fd - np.sum(g * dl)) <= 1e-7 * abs(fd)
