"""The Euler stage kernel's shortcut, checked against oracle roots (CPU).

The kernel accepts the cubic Hermite prediction of lambda (built from F, F' at
t = +-1, four Newton steps on the model) without the confirming third
evaluation when, at t = -1, every population state satisfies |za|, |zb| and
|e_1|/f_1 <= 2^-8 m^2, m = 1 - c^2/W_min^2 (za = (1+al)/(1+be) - 1,
zb = 1/(1+be) - 1 with al, be the relative pressure and density offsets).  Here
the same prediction, restated, is compared with the oracle's root on seeded
states spread over density and pressure in [0.05, 20] and velocities up to
99.9% of the sub-characteristic limit: where the measure holds, the prediction
must move f' = f^eq - lambda d by at most the stop rule's 2 eps max|f|.
"""
import numpy as np
import pytest

from oracle.lattice import Lattice
from oracle.relaxation import entropic_lambda
from oracle.systems import Euler, bregman_sum, equilibrium

EPS = 2.0 ** -52
SKIP = 2.0 ** -8
GAMMA, V = 1.4, 3.2


def hermite_prediction(F1, dF1, Fm, dFm):
    """Root of lambda^2 G(-lambda) = G(1) for the cubic Hermite model of G = F/t^2 on [-1, 1]."""
    G1, Gm, G1p, Gmp = F1, Fm, dF1 - 2 * F1, dFm + 2 * Fm
    cc = 0.25 * (G1p - Gmp)
    dd = 0.25 * ((G1p + Gmp) - (G1 - Gm))
    bb = 0.5 * (G1 - Gm) - dd
    aa = 0.5 * (G1 + Gm) - cc
    lp = np.ones_like(F1)
    for _ in range(4):
        g = aa + lp * (-bb + lp * (cc - dd * lp))
        gp = -bb + lp * (2 * cc - 3 * dd * lp)
        lp = lp - (lp * lp * g - G1) / (2 * lp * g + lp * lp * gp)
    return lp


def sample(rng, n, frac):
    rho = np.exp(rng.uniform(np.log(0.05), np.log(20), n))
    p = np.exp(rng.uniform(np.log(0.05), np.log(20), n))
    lim = frac * V / 2 - np.sqrt(GAMMA * p / rho)
    keep = lim > 0.002
    rho, p, lim = rho[keep], p[keep], lim[keep]
    u = rng.uniform(-1, 1, rho.size) * lim
    v = rng.uniform(-1, 1, rho.size) * lim
    return np.stack([rho, rho * u, rho * v, 0.5 * rho * (u * u + v * v) + p / (GAMMA - 1)])


@pytest.mark.parametrize("frac,seed", [(0.9, 11), (0.99, 12), (0.999, 13)])
def test_skipped_confirmation_stays_within_the_stop_rule(frac, seed):
    lat, sysm = Lattice("D2Q4"), Euler(GAMMA)
    rng = np.random.default_rng(seed)
    U0 = sample(rng, 3000, frac)
    n = U0.shape[1]
    feq0 = equilibrium(lat, sysm, V, U0.reshape(4, 1, n)).reshape(4, 4, n)
    rel = 10.0 ** rng.uniform(-6, -1.5, n)
    f = feq0 + rel * np.abs(feq0) * rng.uniform(-1, 1, feq0.shape)
    U = f.sum(0)
    feq = equilibrium(lat, sysm, V, U.reshape(4, 1, n)).reshape(4, 4, n)
    d = f - feq
    one = np.ones(n)
    F1, dF1, ok1 = bregman_sum(lat, sysm, V, U, feq, d, one)
    Fm, dFm, okm = bregman_sum(lat, sysm, V, U, feq, d, -one)
    lam, fallback = entropic_lambda(lat, sysm, V, U, feq, d)
    rho, vel, p = sysm.primitives(U)
    Wmin = 2 * lat.w * V - np.maximum(np.abs(vel[0]), np.abs(vel[1]))
    m = 1 - GAMMA * p / (rho * Wmin ** 2)
    zlim = np.where((Wmin > 0) & (m > 0), SKIP * m * m, -1.0)
    small = np.ones(n, bool)
    for k in range(4):
        r1, _, p1, valid = sysm.population_state(lat, V, k, feq[k] - d[k])
        al, be = p1 / p - 1, r1 / rho - 1
        za, zb = (al - be) / (1 + be), -be / (1 + be)
        small &= valid & (np.abs(za) <= zlim) & (np.abs(zb) <= zlim) & (np.abs(d[k][0]) <= zlim * feq[k][0])
    use = small & ok1 & okm & ~fallback & (F1 > 0)
    assert use.sum() > 300 and (~use).sum() > 300   # both sides of the threshold are sampled
    lp = hermite_prediction(F1, dF1, Fm, dFm)
    dmax = np.max(np.abs(d), axis=(0, 1))
    fsc = np.maximum(np.max(np.abs(feq), axis=(0, 1)), np.max(np.abs(f), axis=(0, 1)))
    effect = np.abs(lp - lam) * dmax / (2 * EPS * fsc)
    assert effect[use].max() <= 1.0, effect[use].max()


@pytest.mark.parametrize("D,frac,seed", [(1, 0.9, 21), (1, 0.999, 22), (2, 0.9, 23), (2, 0.999, 24)])
def test_skipped_confirmation_shallow_water(D, frac, seed):
    """Shallow water: measure |dh|/h, |e_1|/f_1, |dn|/W at t = -1 against 2^-8 m^2, m = 1 - g h/W_min^2.

    The shallow-water root is itself only determined to about the stop tolerance on both sides (the rounding
    floor of this comparison is ~1 tolerance for every z), so the bound here is 1.5 tolerances.
    """
    from oracle.systems import ShallowWater
    g, V = 9.81, (4.5 if D == 1 else 8.0)
    lat = Lattice("D1Q2" if D == 1 else "D2Q4")
    sysm = ShallowWater(g, D)
    M = D + 1
    rng = np.random.default_rng(seed)
    h = np.exp(rng.uniform(np.log(0.01), np.log(5), 4000))
    W0 = 2 * lat.w * V
    lim = frac * W0 - np.sqrt(g * h)
    keep = lim > 0.002
    h, lim = h[keep], lim[keep]
    n = h.size
    vel = [rng.uniform(-1, 1, n) * lim for _ in range(D)]
    U0 = np.stack([h] + [h * v for v in vel])
    feq0 = equilibrium(lat, sysm, V, U0.reshape(M, 1, n)).reshape(lat.q, M, n)
    rel = 10.0 ** rng.uniform(-6, -1.5, n)
    f = feq0 + rel * np.abs(feq0) * rng.uniform(-1, 1, feq0.shape)
    U = f.sum(0)
    feq = equilibrium(lat, sysm, V, U.reshape(M, 1, n)).reshape(lat.q, M, n)
    d = f - feq
    one = np.ones(n)
    F1, dF1, ok1 = bregman_sum(lat, sysm, V, U, feq, d, one)
    Fm, dFm, okm = bregman_sum(lat, sysm, V, U, feq, d, -one)
    lam, fallback = entropic_lambda(lat, sysm, V, U, feq, d)
    h0 = U[0]
    v0 = [U[1 + j] / h0 for j in range(D)]
    Wmin = W0 - np.max(np.abs(np.array(v0)), axis=0)
    m = 1 - g * h0 / Wmin ** 2
    zlim = np.where((Wmin > 0) & (m > 0), SKIP * m * m, -1.0)
    small = np.ones(n, bool)
    for k in range(lat.q):
        ax, s = lat.axis[k], lat.sign[k]
        h1, v1, valid = sysm.population_state(lat, V, k, feq[k] - d[k])
        Wk = W0 + s * v0[ax]
        small &= valid & (np.abs(h1 - h0) <= zlim * h0) & (np.abs(d[k][0]) <= zlim * feq[k][0])
        small &= np.abs(v1[ax] - v0[ax]) <= zlim * Wk
    use = small & ok1 & okm & ~fallback & (F1 > 0)
    assert use.sum() > 300 and (~use).sum() > 300
    lp = hermite_prediction(F1, dF1, Fm, dFm)
    dmax = np.max(np.abs(d), axis=(0, 1))
    fsc = np.maximum(np.max(np.abs(feq), axis=(0, 1)), np.max(np.abs(f), axis=(0, 1)))
    effect = np.abs(lp - lam) * dmax / (2 * EPS * fsc)
    assert effect[use].max() <= 1.5, effect[use].max()
