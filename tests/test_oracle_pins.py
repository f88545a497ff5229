"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
formulas: printed tables and closed forms come from tests/golden, and the
kinetic entropies are rebuilt in 40-digit arithmetic from their definitions.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from conftest import read_golden
from oracle.exact import SinData, burgers_exact, err_estim, l2_error
from oracle.lattice import Lattice, grid, steps_for_time, time_step, transport
from oracle.relaxation import entropic_lambda, relax_entropic, relax_fixed
from oracle.scheme import Relaxer, brick, composed_step, run, standard_lb_step
from oracle.systems import (Advection, Burgers, Euler, ShallowWater, bregman_sum,
                            equilibrium, kinetic_entropy_sum)
from oracle.diagnostics import diagnostics

D1 = Lattice("D1Q2")
D2 = Lattice("D2Q4")


def rel(a, b):
    return abs(a - b) / abs(b)


def n_from_dx(dx):
    return int(round(1.0 / float(dx)))


# --------------------------------------------------------------------------- tables

def burgers_run(N, mode, V=1.2, T=0.1):
    x, dx = grid(N)
    u0 = SinData(0.0, 1.0)
    sysb = Burgers((1.0,))
    f = equilibrium(D1, sysb, V, u0(x)[None, None, :])
    n = steps_for_time(T, time_step(dx, V))
    fn = run(Relaxer(D1, sysb, V, mode), f, n)
    return l2_error(fn.sum(0)[0, 0], burgers_exact(u0, x, n * time_step(dx, V)), dx)


@pytest.mark.parametrize("row", range(4))
def test_table1_fourth_order(row):
    """Table 1, 4th-order column: Burgers, omega = 2 (Sec. 3.1)."""
    dx, _, e4 = read_golden("table1_burgers_order.txt")[row]
    assert rel(burgers_run(n_from_dx(dx), "fixed"), float(e4)) < 1e-3


@pytest.mark.parametrize("row", range(3))
def test_table1_second_order(row):
    """Table 1, 2nd-order column: (R T(dt/24))^24, i.e. R T(dt/24) steps up to T (Sec. 3.1)."""
    dx, e2, _ = read_golden("table1_burgers_order.txt")[row]
    N = n_from_dx(dx)
    V = 1.2
    x, dx_ = grid(N)
    sysb = Burgers((1.0,))
    u0 = SinData(0.0, 1.0)
    f = equilibrium(D1, sysb, V, u0(x)[None, None, :])
    r = Relaxer(D1, sysb, V)
    dts = time_step(dx_, V) / 24.0
    n = steps_for_time(0.1, dts)
    for _ in range(n):
        f = r(transport(D1, f, 1))
    err = l2_error(f.sum(0)[0, 0], burgers_exact(u0, x, n * dts), dx_)
    assert rel(err, float(e2)) < 1e-3
    # and the composition in blocks of 24 is the same operator
    if n % 24 == 0:
        g = equilibrium(D1, sysb, V, u0(x)[None, None, :])
        for _ in range(n // 24):
            g = standard_lb_step(r, g)
        assert np.array_equal(g, f)


@pytest.mark.parametrize("row", range(3))
def test_table4_entropic(row):
    """Table 4: Burgers with the entropy-limited omega (Sec. 5.1)."""
    dx, e = read_golden("table4_burgers_entropic.txt")[row]
    assert rel(burgers_run(n_from_dx(dx), "entropic"), float(e)) < 1e-3


def sw_run(N, V=1.2, T=5.0 / 16.0):
    x, dx = grid(N)
    sw = ShallowWater(1.0, 1)
    h = 0.5 + 0.2 * np.sin(2 * np.pi * x)
    f = equilibrium(D1, sw, V, np.stack([h, 0 * h])[:, None, :])
    fn = run(Relaxer(D1, sw, V), f, steps_for_time(T, time_step(dx, V)))
    U = fn.sum(0)[:, 0]
    return U[0], U[1] / U[0], dx


@pytest.mark.parametrize("row", range(3))
def test_table2_shallow_water(row):
    """Table 2: shallow water Err-Estim (Sec. 3.2); also pins the node set x_j = j dx."""
    dx, eh, eu = read_golden("table2_sw_errestim.txt")[row]
    N = n_from_dx(dx)
    h1, u1, dx1 = sw_run(N)
    h2, u2, _ = sw_run(2 * N)
    assert rel(err_estim(h1, h2, dx1), float(eh)) < 1e-4
    assert rel(err_estim(u1, u2, dx1), float(eu)) < 1e-4


@pytest.mark.parametrize("row", range(6))
def test_table6_linear_sixth_order_regime(row):
    """Table 6, Scheme I: linear transport at |a| = sqrt(6) V / 12, T = 10 (Sec. 6.2)."""
    dx, e1 = read_golden("table6_linear.txt")[row][:2]
    N = n_from_dx(dx)
    V = 1.2
    a = math.sqrt(6.0) / 12.0 * V
    x, dx_ = grid(N)
    adv = Advection((a,))
    f = equilibrium(D1, adv, V, np.sin(2 * np.pi * x)[None, None, :])
    dt = time_step(dx_, V)
    n = steps_for_time(10.0, dt)
    fn = run(Relaxer(D1, adv, V), f, n)
    err = l2_error(fn.sum(0)[0, 0], np.sin(2 * np.pi * (x - a * n * dt)), dx_)
    assert rel(err, float(e1)) < 1e-3


# ------------------------------------------------------------ linear Fourier symbols

def amplification(a, V, N, m, scheme=1, step=None, omega=2.0):
    """Amplification matrix of the oracle's own step on the Fourier mode m (composed step of the
    given scheme, or ``step(relaxer, f)``)."""
    x = np.arange(N) / N
    e = np.exp(2j * np.pi * m * x)
    r = Relaxer(D1, Advection((a,)), V, omega=omega)
    P = np.zeros((2, 2), complex)
    for c in range(2):
        f = np.zeros((2, 1, 1, N), complex)
        f[c, 0, 0] = e
        g = composed_step(r, f, scheme=scheme) if step is None else step(r, f)
        P[:, c] = g[:, 0, 0, 0] / e[0]
    return P


def trace_polynomial(C, mu):
    C, mu = Fraction(C), Fraction(mu)
    tot = Fraction(0)
    for t in read_golden("appendixA_trace.txt"):
        num = sum(int(c.split(":")[0]) * C ** int(c.split(":")[1]) for c in t[3:])
        tot += (1 if t[1] == "+" else -1) * Fraction(num, int(t[2])) * mu ** int(t[0])
    return float(tot)


@pytest.mark.parametrize("a,V,N,m", [(0.3, 1.0, 40, 3), (0.7, 1.0, 24, 5), (0.95, 1.3, 64, 7),
                                     (-0.5, 1.0, 16, 2), (0.2, 2.0, 50, 9), (0.999, 1.0, 36, 4)])
def test_appendixA_trace_and_det(a, V, N, m):
    """Appendix A: tr of the amplification matrix; Sec. 2.4: det = 1."""
    P = amplification(a, V, N, m)
    C = 24.0 * a / V            # a dt / (kappa dx), kappa = 1
    mu = math.sin(2 * np.pi * m / N)
    assert abs(np.trace(P) - trace_polynomial(C, mu)) < 1e-12
    assert abs(np.linalg.det(P) - 1.0) < 1e-12


def test_jordan_block_at_subcharacteristic_limit():
    """Sec. 2.4: at |a|/V = 1 and xi dx = pi/4 the matrix is [[1, 32 i], [0, 1]]."""
    off = float(dict((r[0], r[1]) for r in read_golden("linear_symbols.txt"))["jordan_offdiag"])
    P = amplification(1.0, 1.0, 8, 1)
    assert np.allclose(P, np.array([[1, 1j * off], [0, 1]]), atol=1e-13, rtol=0)


def test_scheme_I_root_expansion():
    """Sec. 6.2: z1 = exp(-i a xi dt) + i a (24a^4 - 25a^2V^2 + V^4)(xi dt)^5/622080 + (xi dt)^6 a^2(...)/622080."""
    g = dict((r[0], r[1]) for r in read_golden("linear_symbols.txt"))
    a, V = 0.3, 1.0
    poly = 24 * a ** 4 - 25 * a ** 2 * V ** 2 + V ** 4
    c5 = a * poly / float(g["root5_denominator"])
    c6 = a ** 2 * poly / float(g["root6_denominator"])
    im5, re6 = [], []
    for N in (754, 1508):            # xi dt ~ 0.2, 0.1
        xdt = 2 * np.pi / N * 24 / V
        z = np.linalg.eigvals(amplification(a, V, N, 1))
        ref = np.exp(-1j * a * xdt)
        z1 = z[np.argmin(np.abs(z - ref))]
        im5.append((z1 - ref).imag / xdt ** 5)
        re6.append((z1 - ref).real / xdt ** 6)
    # Richardson on the O(xi dt)^2 correction
    assert rel((4 * im5[1] - im5[0]) / 3, c5) < 2e-4
    assert rel((4 * re6[1] - re6[0]) / 3, c6) < 2e-3


def _root_coefficients(a, V, scheme, Ns=(192, 384, 768)):
    """Fifth- and sixth-order coefficients of z1 - exp(-i a xi dt) by Richardson on the (xi dt)^2
    term (the fifth-order one from the two finer grids, the sixth-order one, whose difference is
    smaller, from the two coarser ones) and the largest modulus of the other root, from the oracle's
    amplification matrices."""
    im5, re6, z2 = [], [], 0.0
    for N in Ns:
        xdt = 2 * np.pi / N * 24 / V
        z = np.linalg.eigvals(amplification(a, V, N, 1, scheme))
        ref = np.exp(-1j * a * xdt)
        i1 = int(np.argmin(np.abs(z - ref)))
        im5.append((z[i1] - ref).imag / xdt ** 5)
        re6.append((z[i1] - ref).real / xdt ** 6)
        z2 = max(z2, float(abs(z[1 - i1])))
    return (4 * im5[2] - im5[1]) / 3, (4 * re6[1] - re6[0]) / 3, z2


@pytest.mark.parametrize("a", [0.3, 0.45])
def test_scheme_II_root_expansion(a):
    """Sec. 6.2, Scheme II: z2 = 0, z1 has Scheme I's fifth- and sixth-order terms."""
    g = dict((r[0], r[1]) for r in read_golden("linear_symbols.txt"))
    V = 1.0
    poly = 24 * a ** 4 - 25 * a ** 2 * V ** 2 + V ** 4
    c5, c6, z2 = _root_coefficients(a, V, 2)
    assert z2 < 1e-14
    assert rel(c5, a * poly / float(g["root5_denominator"])) < 5e-4
    assert rel(c6, a ** 2 * poly / float(g["root6_denominator"])) < 5e-4


@pytest.mark.parametrize("a", [math.sqrt(6.0) / 12.0, 0.3, 0.45])
def test_scheme_III_root_expansion(a):
    """Sec. 6.2, Scheme III: z2 = 0, Scheme I's fifth-order term and the sixth-order term
    a^2 (63 a^4 - 65 a^2 V^2 + 2 V^4) / 1244160.  At |a| = sqrt(6) V / 12 the fifth-order
    term vanishes and the sixth-order one is all that is left (the scheme stays fifth order there,
    Table 6).  Placing the projections between the bricks only moves this coefficient by 1-3 %."""
    row = [r for r in read_golden("linear_symbols.txt") if r[0] == "scheme3_root6"][0]
    k4, k2, k0, den = (float(v) for v in row[1:])
    V = 1.0
    poly = 24 * a ** 4 - 25 * a ** 2 * V ** 2 + V ** 4
    want6 = a ** 2 * (k4 * a ** 4 + k2 * a ** 2 * V ** 2 + k0 * V ** 4) / den
    c5, c6, z2 = _root_coefficients(a, V, 3)
    assert z2 < 1e-14
    assert rel(c6, want6) < 5e-4, (c6, want6)
    if abs(poly) > 1e-12:
        assert rel(c5, a * poly / 622080.0) < 5e-4
    else:
        assert abs(c5) < 1e-3 * abs(want6)


def test_scheme_A_symbol_closed_form():
    """Sec. 6.3, Scheme (A): one step R_omega T(dt), dt = kappa dx / V, on linear D1Q2.

    Hand derivation: T(dt) multiplies the Fourier mode of f_+ by c = exp(-i theta) and that of
    f_- by conj(c) (pull shift by one cell, theta = xi dx); R_omega = (1 - omega) I + omega E with
    E = [[w+, w+], [w-, w-]], w+- = (1 +- a/V)/2 (f^eq_+- = w+- u).  So
        A = [[(1 - omega + omega w+) c, omega w+ conj(c)], [omega w- c, (1 - omega + omega w-) conj(c)]],
    det A = 1 - omega, tr A = (2 - omega) cos theta - i omega (a/V) sin theta."""
    from oracle.scheme import scheme_A_step
    for a, V, omega, N, m in ((0.3, 1.0, 1.93, 40, 3), (-0.7, 1.3, 1.5, 24, 5), (0.9, 1.0, 2.0, 64, 7)):
        P = amplification(a, V, N, m, step=scheme_A_step, omega=omega)
        th = 2 * np.pi * m / N
        c = np.exp(-1j * th)
        wp, wm = 0.5 * (1 + a / V), 0.5 * (1 - a / V)
        want = np.array([[(1 - omega + omega * wp) * c, omega * wp * np.conj(c)],
                         [omega * wm * c, (1 - omega + omega * wm) * np.conj(c)]])
        assert np.max(np.abs(P - want)) < 1e-14
        assert abs(np.linalg.det(P) - (1 - omega)) < 1e-14
        assert abs(np.trace(P) - ((2 - omega) * np.cos(th) - 1j * omega * a / V * np.sin(th))) < 1e-14


def test_scheme_B_symbol_closed_form():
    """Sec. 6.3, Scheme (B): R_1 T(dt/4) R_2 T(dt/2) R_2 T(dt/4), dt = 4 kappa dx / V, linear D1Q2.

    Hand derivation (notation of the Scheme (A) test, sigma_k = c^k w+ + conj(c)^k w- =
    cos k theta - i (a/V) sin k theta, s = sigma_1): the final projection makes the matrix
    w r^T with w = (w+, w-) and the row r^T = 1^T T(1) R_2 T(2) R_2 T(1),
        r = (2 (2 s sigma_2 - sigma_3) c - (2 s - c) c^3,  2 (2 s sigma_2 - sigma_3) conj(c) - (2 s - conj(c)) conj(c)^3),
    so det = 0 and the non-zero root is tr = 4 s^2 sigma_2 - 4 s sigma_3 + sigma_4 (c^4 at a = V: a
    translation by four cells).  Projecting first instead (T(1) R_2 T(2) R_2 T(1) R_1) has the same
    roots but a matrix whose rows are multiples of 1^T: the full matrix tells the two apart."""
    from oracle.scheme import scheme_B_step
    for a, V, N, m in ((0.3, 1.0, 40, 3), (-0.7, 1.3, 24, 5), (0.95, 1.0, 64, 7), (1.0, 1.0, 16, 1)):
        P = amplification(a, V, N, m, step=scheme_B_step)
        th = 2 * np.pi * m / N
        c, cb = np.exp(-1j * th), np.exp(1j * th)
        wp, wm = 0.5 * (1 + a / V), 0.5 * (1 - a / V)
        sig = lambda k: np.cos(k * th) - 1j * (a / V) * np.sin(k * th)
        s = sig(1)
        b = 2 * (2 * s * sig(2) - sig(3))
        r = np.array([b * c - (2 * s - c) * c ** 3, b * cb - (2 * s - cb) * cb ** 3])
        want = np.outer([wp, wm], r)
        assert np.max(np.abs(P - want)) < 1e-14
        assert abs(np.trace(P) - (4 * s * s * sig(2) - 4 * s * sig(3) + sig(4))) < 1e-14
        if a == V:
            assert abs(np.trace(P) - c ** 4) < 1e-14


# ------------------------------------------------------------- transport and symmetry

def test_transport_is_the_pull_shift():
    """eq. transportPhase: f_k(x) <- f_k(x - s c_k dx), written as an index loop."""
    rng = np.random.default_rng(1)
    f = rng.standard_normal((4, 2, 5, 7))
    for s in (1, 2, -1, -4, 9):
        g = transport(D2, f, s)
        for k in range(4):
            cx, cy = D2.c[k]
            for y in range(5):
                for xx in range(7):
                    assert g[k, :, y, xx].tolist() == f[k, :, (y - s * cy) % 5, (xx - s * cx) % 7].tolist()


def test_exact_translation_bitwise():
    """a = V: f_- = 0 and R is the identity, so u(t_n) is u0 moved by V t_n / dx = 24 n cells."""
    N = 96
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(N)
    V = 1.0
    adv = Advection((1.0,))
    f = equilibrium(D1, adv, V, u0[None, None, :])
    for mode in ("fixed", "entropic"):
        g = run(Relaxer(D1, adv, V, mode), f, 3)
        assert np.array_equal(g.sum(0)[0, 0], np.roll(u0, 72))


def smooth_state(sysname, shape, rng, amp=0.05):
    """A near-equilibrium state with random smooth perturbations (test data only)."""
    ny, nx = shape
    y, x = np.meshgrid(np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def field():
        out = np.zeros(shape)
        for _ in range(3):
            kx, ky = rng.integers(1, 4, size=2)
            out += rng.uniform(-1, 1) * np.sin(2 * np.pi * (kx * x + (ky * y if ny > 1 else 0)) + rng.uniform(0, 6))
        return amp * out / max(np.max(np.abs(out)), 1e-300)

    if sysname == "burgers1d":
        return D1, Burgers((1.0,)), 1.5, (0.4 + field())[None]
    if sysname == "sw1d":
        h = 1.0 + field()
        return D1, ShallowWater(9.81, 1), 4.5, np.stack([h, h * field()])
    if sysname == "sw2d":
        h = 1.0 + field()
        return D2, ShallowWater(9.81, 2), 8.0, np.stack([h, h * field(), h * field()])
    if sysname == "euler2d":
        rho = 1.0 + field()
        uu, vv, p = field(), field(), 1.0 + field()
        E = 0.5 * rho * (uu ** 2 + vv ** 2) + p / 0.4
        return D2, Euler(1.4, 2), 3.2, np.stack([rho, rho * uu, rho * vv, E])
    if sysname == "burgers2d":
        return D2, Burgers((1.0, 0.6)), 2.0, (0.3 + field())[None]
    raise ValueError(sysname)


SYSTEMS = ["burgers1d", "sw1d", "sw2d", "euler2d", "burgers2d"]


def shape_of(name):
    return (1, 48) if name.endswith("1d") else (12, 10)


@pytest.mark.parametrize("name", SYSTEMS)
@pytest.mark.parametrize("mode", ["fixed", "entropic"])
def test_time_symmetry_of_the_brick(name, mode):
    """eq. symmetryCondition: psi(-dt) psi(dt) = Id, with R = R_2 or the entropic R (Sec. 4)."""
    rng = np.random.default_rng(3)
    lat, sys, V, u = smooth_state(name, shape_of(name), rng)
    f = equilibrium(lat, sys, V, u)
    f = f + 1e-3 * rng.standard_normal(f.shape) * np.abs(f).max()   # off equilibrium
    f = f - (f.sum(0) - u)[None] / lat.q
    r = Relaxer(lat, sys, V, mode)
    g = brick(r, brick(r, f, 4), -4)
    assert np.max(np.abs(g - f)) <= 1e-13 * np.max(np.abs(f))
    # psi(0) = Id: the brick with zero transport is R R
    assert np.max(np.abs(brick(r, f, 0) - f)) <= 1e-13 * np.max(np.abs(f))


@pytest.mark.parametrize("name", SYSTEMS)
def test_entropic_relaxation_is_an_involution_and_conserves(name):
    """Sec. 4: R_{omega(R f)} R_{omega(f)} f = f; R conserves u and Sigma at every node."""
    rng = np.random.default_rng(4)
    lat, sys, V, u = smooth_state(name, shape_of(name), rng)
    f = transport(lat, equilibrium(lat, sys, V, u), 1)
    g, om, fb = relax_entropic(lat, sys, V, f, return_info=True)
    assert not fb.any()
    h = relax_entropic(lat, sys, V, g)
    scale = np.max(np.abs(f))
    assert np.max(np.abs(h - f)) <= 1e-13 * scale
    assert np.max(np.abs(g.sum(0) - f.sum(0))) <= 8 * np.finfo(float).eps * np.max(np.abs(f).sum(0))
    s0, _ = kinetic_entropy_sum(lat, sys, V, f)
    s1, _ = kinetic_entropy_sum(lat, sys, V, g)
    assert np.max(np.abs(s1 - s0)) <= 1e-13 * np.max(np.abs(s0))


@pytest.mark.parametrize("name", ["burgers1d", "sw1d", "euler2d"])
def test_run_conserves_mass_and_bounds_entropy(name):
    """Sec. 4: transport and relaxation conserve sum_x u and sum_x Sigma; sum_x S(u_n) <= sum_x S(u_0)."""
    rng = np.random.default_rng(5)
    lat, sys, V, u = smooth_state(name, shape_of(name), rng)
    f = equilibrium(lat, sys, V, u)
    d0 = diagnostics(lat, sys, V, f)
    recs = []
    run(Relaxer(lat, sys, V, "entropic"), f, 3, callback=lambda i, g: recs.append(diagnostics(lat, sys, V, g)))
    for d in recs:
        for m0, m1 in zip(d0["mass"], d["mass"]):
            assert abs(m1 - m0) <= 1e-12 * max(abs(m0), 1.0)
        assert abs(d["micro_entropy"] - d0["micro_entropy"]) <= 1e-13 * abs(d0["micro_entropy"]) * 20
        assert d["macro_entropy"] <= d0["micro_entropy"] + 1e-13 * abs(d0["micro_entropy"])
    assert abs(d0["micro_entropy"] - d0["macro_entropy"]) <= 1e-13 * abs(d0["macro_entropy"])


def test_linear_quadratic_entropy_gives_omega_two():
    """Proposition of Sec. 4: linear flux + quadratic entropies => R_2 conserves Sigma, so omega = 2."""
    rng = np.random.default_rng(6)
    for lat, a in ((D1, (0.4,)), (D2, (0.2, -0.3))):
        adv = Advection(a)
        f = rng.standard_normal((lat.q, 1, 3, 17))
        g, om, fb = relax_entropic(lat, adv, 1.0, f, return_info=True)
        assert np.max(np.abs(om - 2.0)) < 1e-12
        assert np.max(np.abs(g - relax_fixed(lat, adv, 1.0, f, 2.0))) < 1e-14


# ----------------------------------------------- brute force of the kinetic entropies

mp.mp.dps = 40


def mp_model(name, lat, sys, V):
    """Flux, entropy, entropy flux of each system in mpmath, straight from Sec. 1-6."""
    V = mp.mpf(V)
    if isinstance(sys, Burgers):
        b = [mp.mpf(x) for x in sys.b]
        flux = lambda U, j: [b[j] * U[0] ** 2 / 2]
        S = lambda U: U[0] ** 2 / 2
        G = lambda U, j: b[j] * U[0] ** 3 / 3
        v = lambda U: [U[0]]
    elif isinstance(sys, ShallowWater):
        g = mp.mpf(sys.g)
        d = sys.d

        def flux(U, j):
            h = U[0]
            vel = [U[1 + i] / h for i in range(d)]
            out = [U[1 + j]] + [U[1 + j] * vel[i] for i in range(d)]
            out[1 + j] += g * h ** 2 / 2
            return out
        S = lambda U: sum(U[1 + i] ** 2 for i in range(d)) / (2 * U[0]) + g * U[0] ** 2 / 2
        G = lambda U, j: (S(U) + g * U[0] ** 2 / 2) * U[1 + j] / U[0]
        v = lambda U: [g * U[0] - sum((U[1 + i] / U[0]) ** 2 for i in range(d)) / 2] + [U[1 + i] / U[0] for i in range(d)]
    else:
        gm = mp.mpf(sys.gamma)
        d = sys.d

        def prim(U):
            rho = U[0]
            vel = [U[1 + i] / rho for i in range(d)]
            p = (gm - 1) * (U[1 + d] - rho * sum(c * c for c in vel) / 2)
            return rho, vel, p

        def flux(U, j):
            rho, vel, p = prim(U)
            out = [U[1 + j]] + [U[1 + j] * vel[i] for i in range(d)] + [vel[j] * (U[1 + d] + p)]
            out[1 + j] += p
            return out

        def S(U):
            rho, vel, p = prim(U)
            return -rho * (mp.log(p) - gm * mp.log(rho)) / (gm - 1)
        G = lambda U, j: S(U) * U[1 + j] / U[0]

        def v(U):
            rho, vel, p = prim(U)
            s = mp.log(p) - gm * mp.log(rho)
            beta = rho / p
            return [(gm - s) / (gm - 1) - beta * sum(c * c for c in vel) / 2] + [beta * c for c in vel] + [-beta]
    w = mp.mpf(1) / lat.q

    def feq(k, U):
        fl = flux(U, lat.axis[k])
        return [w * U[m] + lat.sign[k] * fl[m] / (2 * V) for m in range(len(U))]

    def s_k(k, x, guess):
        """s_k(x) = v(U).x - s_k^*(v(U)), f_k^eq(U) = x, s_k^* = w S^* + sigma G^{n,*}/(2V) (eq. transformationEntropyFlux)."""
        M = len(x)
        U = mp.findroot(lambda *Us: [a - b for a, b in zip(feq(k, list(Us)), x)], guess)
        U = [U[i] for i in range(M)] if isinstance(U, mp.matrix) else [U]
        vv = v(U)
        Sstar = sum(a * b for a, b in zip(vv, U)) - S(U)
        n = lat.axis[k]
        Gstar = sum(a * b for a, b in zip(flux(U, n), vv)) - G(U, n)
        sstar = w * Sstar + lat.sign[k] * Gstar / (2 * V)
        return sum(a * b for a, b in zip(vv, x)) - sstar

    return feq, s_k, S


@pytest.mark.parametrize("name", SYSTEMS)
def test_bregman_form_and_omega_against_brute_force(name):
    """F(t) equals Sigma(f^eq + t d) - S(u) built from the definitions; omega solves eq. variableOmegaProblem."""
    rng = np.random.default_rng(7)
    lat, sys, V, u = smooth_state(name, (1, 3) if lat_is_1d(name) else (1, 3), rng)
    u = u.reshape(u.shape[0], -1)[:, :2]
    feq = equilibrium(lat, sys, V, u)
    d = 3e-3 * rng.standard_normal(feq.shape) * np.abs(feq).max()
    d = d - d.mean(axis=0, keepdims=True)           # sum_k d_k = 0
    mfeq, s_k, S = mp_model(name, lat, sys, V)
    lam, fb = entropic_lambda(lat, sys, V, u, feq, d)
    assert not fb.any()
    for c in range(u.shape[1]):
        U0 = [mp.mpf(float(a)) for a in u[:, c]]
        fe = [[mp.mpf(float(a)) for a in feq[k, :, c]] for k in range(lat.q)]
        dd = [[mp.mpf(float(a)) for a in d[k, :, c]] for k in range(lat.q)]

        def sigma(t):
            return sum(s_k(k, [fe[k][m] + t * dd[k][m] for m in range(len(U0))], U0) for k in range(lat.q))

        for t in (1.0, -0.7, 1.3):
            F, _, ok = bregman_sum(lat, sys, V, u[:, c:c + 1], feq[:, :, c:c + 1], d[:, :, c:c + 1], np.array([t]))
            ref = sigma(mp.mpf(t)) - S(U0)
            assert ok[0]
            assert rel(F[0], float(ref)) < 1e-9
        S1 = sigma(mp.mpf(1))
        root = mp.findroot(lambda L: sigma(-L) - S1, mp.mpf(1))
        assert abs(lam[c] - float(root)) < 1e-10


def lat_is_1d(name):
    return name.endswith("1d")


def test_shallow_water_branch_matches_polynomial_roots():
    """Example "Shallow water": the population state's normal velocity is the extreme real root of the cubic."""
    rng = np.random.default_rng(8)
    for lat, d in ((D1, 1), (D2, 2)):
        sw = ShallowWater(9.81, d)
        V = 4.5 if d == 1 else 8.0
        for trial in range(20):
            h = rng.uniform(0.8, 1.2)
            vel = rng.uniform(-0.3, 0.3, size=d)
            u = np.concatenate([[h], h * vel])[:, None]
            feq = equilibrium(lat, sw, V, u)
            for k in range(lat.q):
                x = feq[k] + (1e-2 if d == 1 else 1e-3) * rng.standard_normal(feq[k].shape)
                hp, velp, ok = sw.population_state(lat, V, k, x)
                assert ok[0]
                n, s = lat.axis[k], lat.sign[k]
                W0 = 2 * lat.w * V
                x1, xn = x[0, 0], x[1 + n, 0]
                # (xn - x1 z)(W0 + s z)^2 - s g V x1^2 expanded by numpy.polymul
                poly = np.polysub(np.polymul([-x1, xn], np.polymul([s, W0], [s, W0])), [s * 9.81 * V * x1 ** 2])
                r = np.roots(poly)
                r = r[np.abs(r.imag) < 1e-9].real
                want = r.max() if s > 0 else r.min()
                assert abs(velp[n, 0] - want) < 1e-12
                # round trip f^eq(U_k) = x
                U = np.concatenate([[hp[0]], hp[0] * velp[:, 0]])[:, None]
                assert np.max(np.abs(equilibrium(lat, sw, V, U)[k] - x)) < 1e-14


def test_euler_branch_round_trip_and_other_root_inadmissible():
    """Euler population state: f^eq(U_k) = x, and the discarded root violates rho W^2 > gamma p.

    Both candidates come from the equilibrium's definition, not from the oracle's quadratic:
    with z the normal velocity, W = 2wV + sigma z, the relations x_1 = rho W / (2V),
    x_n = z x_1 + sigma p / (2V), x_t = u_t x_1, x_E = (E W + sigma z p) / (2V) give
    p = 2 sigma V (x_n - z x_1), rho W = 2 V x_1, and the energy relation
    p W / (gamma - 1) + V x_1 (z^2 + u_t^2) + sigma z p - 2 V x_E = 0, a quadratic in z
    multiplied out here with numpy's polynomial arithmetic."""
    from numpy.polynomial import Polynomial as Pn
    rng = np.random.default_rng(9)
    eu = Euler(1.4, 2)
    gm, V = 1.4, 3.2
    W0 = 2 * D2.w * V
    for trial in range(20):
        rho, p = rng.uniform(0.9, 1.1, size=2)
        vel = rng.uniform(-0.1, 0.1, size=2)
        E = 0.5 * rho * vel @ vel + p / 0.4
        u = np.array([rho, rho * vel[0], rho * vel[1], E])[:, None]
        feq = equilibrium(D2, eu, V, u)
        for k in range(4):
            x = feq[k] + 1e-3 * rng.standard_normal(feq[k].shape)
            rp, velp, pp, ok = eu.population_state(D2, V, k, x)
            assert ok[0]
            Ek = 0.5 * rp * np.sum(velp ** 2, axis=0) + pp / 0.4
            U = np.concatenate([rp, rp * velp[0], rp * velp[1], Ek])[:, None]
            assert np.max(np.abs(equilibrium(D2, eu, V, U)[k] - x)) < 1e-14
            n, sg = D2.axis[k], D2.sign[k]
            x1, xn, xt, xE = x[0, 0], x[1 + n, 0], x[2 - n, 0], x[3, 0]
            z = Pn([0.0, 1.0])
            Wz = W0 + sg * z
            pz = 2 * sg * V * (xn - z * x1)
            quad = pz * Wz / (gm - 1) + V * x1 * (z * z + (xt / x1) ** 2) + sg * z * pz - 2 * V * xE
            roots = quad.roots()
            assert np.all(np.abs(np.imag(roots)) == 0)
            roots = np.real(roots)
            i = int(np.argmin(np.abs(roots - velp[n, 0])))
            assert abs(roots[i] - velp[n, 0]) < 1e-12
            zo = roots[1 - i]
            Wo, po = W0 + sg * zo, 2 * sg * V * (xn - zo * x1)
            rho_o = 2 * V * x1 / Wo
            admissible = (Wo > 0) and (po > 0) and (rho_o > 0) and (rho_o * Wo ** 2 > gm * po)
            assert not admissible, (k, zo, Wo, po, rho_o)


def test_newton_root_equals_dichotomy():
    """The root finder gives the same lambda as a plain dichotomy (Sec. 5.1 uses one)."""
    rng = np.random.default_rng(10)
    lat, sys, V, u = smooth_state("sw1d", (1, 16), rng)
    u = u.reshape(2, -1)
    feq = equilibrium(lat, sys, V, u)
    d = 2e-3 * rng.standard_normal(feq.shape)
    d -= d.mean(axis=0, keepdims=True)
    lam, _ = entropic_lambda(lat, sys, V, u, feq, d)
    F1, _, _ = bregman_sum(lat, sys, V, u, feq, d, np.ones(u.shape[1]))
    lo, hi = np.zeros(u.shape[1]), np.full(u.shape[1], 4.0)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        Fm, _, ok = bregman_sum(lat, sys, V, u, feq, d, -mid)
        up = ~ok | (Fm > F1)
        hi = np.where(up, mid, hi)
        lo = np.where(up, lo, mid)
    # equal up to the resolution of f^eq - lambda d
    assert np.max(np.abs(lam - 0.5 * (lo + hi)) * np.abs(d).max(axis=(0, 1))) < 1e-15


def test_fallback_when_outside_the_convexity_domain():
    """Reading for the silent case: f outside the domain => omega = 1 (projection), flagged."""
    sysb = Burgers((1.0,))
    V = 1.0
    u = np.array([[0.2]])
    feq = equilibrium(D1, sysb, V, u)
    f = feq.copy()
    f[0, 0, 0] -= 0.4            # f_+ = -0.3: 1 + 4 f_+ / V < 0
    f[1, 0, 0] += 0.4
    g, om, fb = relax_entropic(D1, sysb, V, f, return_info=True)
    assert fb.all() and np.allclose(om, 1.0)
    assert np.allclose(g, feq)


# ----------------------------------------------------------------------- order

def test_fourth_order_convergence_entropic_burgers():
    """Measured order ~4 (Sec. 3.1 / 5.1): smooth Burgers family with V = 2, T = 0.2, entropic omega."""
    V, T = 2.0, 0.2
    u0 = SinData(0.5, 0.25, ((2, 0.01, 0.3), (3, 0.008, 1.1)))
    errs = []
    Ns = (120, 240, 480, 960)
    for N in Ns:
        x, dx = grid(N)
        sysb = Burgers((1.0,))
        f = equilibrium(D1, sysb, V, u0(x)[None, None, :])
        dt = time_step(dx, V)
        n = steps_for_time(T, dt)
        fn = run(Relaxer(D1, sysb, V, "entropic"), f, n)
        errs.append(l2_error(fn.sum(0)[0, 0], burgers_exact(u0, x, n * dt), dx))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert -4.4 < slope < -3.6, (errs, slope)


def test_fourth_order_self_convergence_entropic_shallow_water():
    """Err-Estim slope (Sec. 3.2, Table 2's definition: the N run against every other node of the
    2N run) of the entropic scheme on Table 2's shallow-water setting: g = 1, V = 1.2,
    h0 = 1/2 + sin(2 pi x)/5, u0 = 0, T = 5/16, error on the velocity u = hu / h."""
    V, T = 1.2, 5.0 / 16.0
    sysw = ShallowWater(1.0, 1)
    vel, dxs = {}, {}
    for N in (128, 256, 512, 1024):
        x, dx = grid(N)
        h = 0.5 + 0.2 * np.sin(2 * np.pi * x)
        f = equilibrium(D1, sysw, V, np.stack([h, 0.0 * h])[:, None, :])
        u = run(Relaxer(D1, sysw, V, "entropic"), f, steps_for_time(T, time_step(dx, V))).sum(0)[:, 0]
        vel[N], dxs[N] = u[1] / u[0], dx
    Ns = (128, 256, 512)
    errs = [err_estim(vel[N], vel[2 * N], dxs[N]) for N in Ns]
    slope = -np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    assert 3.6 < slope < 4.6, (errs, slope)


def test_fourth_order_self_convergence_entropic_euler_d2q4():
    """Err-Estim slope of the entropic D2Q4^4 Euler scheme (gamma = 1.4, V = 3.2) on smooth periodic
    data that vary along x only, on a strip three nodes high (every population of the 2D lattice
    moves and relaxes; refinement along x costs N, not N^2): rho = 1 + sin(2 pi x)/10,
    u = cos(2 pi x)/10, v = sin(2 pi x + 1)/20, p = 1 + cos(2 pi x)/10, to T = 48 / (32 V)."""
    V = 3.2
    eu = Euler(1.4, 2)
    out, dxs = {}, {}
    for N in (64, 128, 256, 512):
        x = np.arange(N) / N
        rho, uu = 1 + 0.1 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * x)
        vv, p = 0.05 * np.sin(2 * np.pi * x + 1.0), 1 + 0.1 * np.cos(2 * np.pi * x)
        U = np.stack([rho, rho * uu, rho * vv, 0.5 * rho * (uu ** 2 + vv ** 2) + p / 0.4])
        U = np.repeat(U[:, None, :], 3, axis=1)
        f = equilibrium(D2, eu, V, U)
        dx = 1.0 / N
        n = steps_for_time(48.0 / (32 * V), time_step(dx, V))
        out[N], dxs[N] = run(Relaxer(D2, eu, V, "entropic"), f, n).sum(0)[:, 0, :], dx
    Ns = (64, 128, 256)
    for m in range(4):
        errs = [err_estim(out[N][m], out[2 * N][m], dxs[N]) for N in Ns]
        slope = -np.polyfit(np.log(Ns), np.log(errs), 1)[0]
        assert 3.6 < slope < 4.6, (m, errs, slope)


# ------------------------------------------------------- projection variants (Sec. 6.1)

def _table5_run(N, init, scheme):
    V = 1.2
    x, dx = grid(N)
    u0 = SinData(0.0, 1.0)
    sysb = Burgers((1.0,))
    u = u0(x)[None, None, :]
    # off-equilibrium initialisation of Sec. 6.2: (f+, f-)(0) = (1/4, 3/4) u0
    f = equilibrium(D1, sysb, V, u) if init == "eq" else np.stack([0.25 * u, 0.75 * u])
    dt = time_step(dx, V)
    n = steps_for_time(0.1, dt)
    fn = run(Relaxer(D1, sysb, V, "fixed"), f, n, scheme=scheme)
    return l2_error(fn.sum(0)[0, 0], burgers_exact(u0, x, n * dt), dx)


@pytest.mark.parametrize("row", [0, 1, 4, 5])
@pytest.mark.parametrize("scheme", [1, 2])
def test_table5_schemes_I_II(row, scheme):
    """Table 5: Schemes I and II, initial data at and off equilibrium (Sec. 6.2)."""
    r = read_golden("table5_schemes_burgers.txt")[row]
    init, dx = r[0], r[1]
    assert rel(_table5_run(n_from_dx(dx), init, scheme), float(r[1 + scheme])) < 1e-3


def test_table5_scheme_III_at_equilibrium_N800():
    """Table 5, Scheme III (R_1 after every brick), data at equilibrium, dx = 1.25e-3.

    Only this row of the Scheme III column reproduces under the reading used here;
    the N = 500 row (3.221e-6 vs 3.246e-6) and Table 6's Scheme III column do not.
    """
    r = read_golden("table5_schemes_burgers.txt")[1]
    assert rel(_table5_run(n_from_dx(r[1]), "eq", 3), float(r[4])) < 1e-3


@pytest.mark.parametrize("row", range(3))
def test_table6_scheme_II(row):
    """Table 6, Scheme II: the final projection does not change the conserved moment."""
    dx, _, e2 = read_golden("table6_linear.txt")[row][:3]
    N = n_from_dx(dx)
    V = 1.2
    a = math.sqrt(6.0) / 12.0 * V
    x, dx_ = grid(N)
    adv = Advection((a,))
    f = equilibrium(D1, adv, V, np.sin(2 * np.pi * x)[None, None, :])
    dt = time_step(dx_, V)
    n = steps_for_time(10.0, dt)
    fn = run(Relaxer(D1, adv, V), f, n, scheme=2)
    assert rel(l2_error(fn.sum(0)[0, 0], np.sin(2 * np.pi * (x - a * n * dt)), dx_), float(e2)) < 1e-3
