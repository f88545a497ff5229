"""40-digit brute force of the entropic relaxation far from equilibrium (Sec. 4, eq. variableOmegaProblem).

The stage inputs are drawn exactly as the GPU parity tests of far-from-equilibrium passes draw
them (relative offsets of f from f^eq of 1 % to 30 %).  For every system the population state
U_k of a population value x is found here from the definition of the equilibrium,
f_k^eq(U) = w U + sigma phi^n(U) / (2V) (Sec. 1.2), eliminated by hand into one polynomial in
the normal velocity (Euler: quadratic; shallow water: cubic; Burgers: quadratic in u) whose
real roots mpmath finds; the admissible root is the one where the kinetic entropy is convex
(W' > 0 and the sub-characteristic condition).  The kinetic entropies are then built from
their definition s_k(x) = v(U_k).x - s_k^*(v(U_k)), s_k^* = w S^* + sigma G^{n,*}/(2V)
(eq. transformationEntropyFlux), with S^* = v.U - S and G^{n,*} = v.phi^n - G^n.  None of
the oracle's increment formulas is used.

Checked against the oracle, node by node:
  * where the oracle finds a root: the 40-digit root of Sigma(f^eq - L d) = Sigma(f) equals
    the oracle's lambda to within its stop rule (|dlambda| max|d| <= 4 eps max|f|);
  * where the oracle falls back to omega = 1: either some population of f itself has no
    admissible state, or the populations of f^eq - L d leave the convexity domain at some
    L_edge with Sigma(f^eq - L d) still below Sigma(f) there, so no root lies inside
    the domain (Sigma(f^eq - L d) increases with L on it: F is convex with its minimum at 0).
"""
import mpmath as mp
import numpy as np
import pytest

from oracle.lattice import Lattice
from oracle.relaxation import relax_entropic
from oracle.systems import Burgers, Euler, ShallowWater, equilibrium
from paper_2403_13406_amd import workloads as W

mp.mp.dps = 40
EPS = np.finfo(float).eps


class Model:
    """Flux, entropy pair and population-state inversion of one system, in mpmath."""

    def __init__(self, lat, sys, V):
        self.lat, self.sys, self.V = lat, sys, mp.mpf(V)
        self.w = mp.mpf(1) / lat.q
        self.W0 = 2 * self.w * self.V

    # -- the system (Sec. 1.1, the examples of Sec. 1.2, Sec. 6.3)
    def flux(self, U, j):
        s = self.sys
        if isinstance(s, Burgers):
            return [mp.mpf(s.b[j]) * U[0] ** 2 / 2]
        d = s.d
        if isinstance(s, ShallowWater):
            g = mp.mpf(s.g)
            h = U[0]
            out = [U[1 + j]] + [U[1 + j] * U[1 + i] / h for i in range(d)]
            out[1 + j] += g * h ** 2 / 2
            return out
        rho, vel, p = self.prim(U)
        out = [U[1 + j]] + [U[1 + j] * vel[i] for i in range(d)] + [vel[j] * (U[1 + d] + p)]
        out[1 + j] += p
        return out

    def prim(self, U):
        d, gm = self.sys.d, mp.mpf(self.sys.gamma)
        rho = U[0]
        vel = [U[1 + i] / rho for i in range(d)]
        return rho, vel, (gm - 1) * (U[1 + d] - rho * sum(c * c for c in vel) / 2)

    def S(self, U):
        s = self.sys
        if isinstance(s, Burgers):
            return U[0] ** 2 / 2
        if isinstance(s, ShallowWater):
            return sum(U[1 + i] ** 2 for i in range(s.d)) / (2 * U[0]) + mp.mpf(s.g) * U[0] ** 2 / 2
        gm = mp.mpf(s.gamma)
        rho, vel, p = self.prim(U)
        return -rho * (mp.log(p) - gm * mp.log(rho)) / (gm - 1)

    def G(self, U, j):
        s = self.sys
        if isinstance(s, Burgers):
            return mp.mpf(s.b[j]) * U[0] ** 3 / 3
        if isinstance(s, ShallowWater):
            return (self.S(U) + mp.mpf(s.g) * U[0] ** 2 / 2) * U[1 + j] / U[0]
        return self.S(U) * U[1 + j] / U[0]

    def v(self, U):
        s = self.sys
        if isinstance(s, Burgers):
            return [U[0]]
        if isinstance(s, ShallowWater):
            h = U[0]
            vel = [U[1 + i] / h for i in range(s.d)]
            return [mp.mpf(s.g) * h - sum(c * c for c in vel) / 2] + vel
        gm = mp.mpf(s.gamma)
        rho, vel, p = self.prim(U)
        ent = mp.log(p) - gm * mp.log(rho)
        beta = rho / p
        return [(gm - ent) / (gm - 1) - beta * sum(c * c for c in vel) / 2] + [beta * c for c in vel] + [-beta]

    def feq(self, k, U):
        fl = self.flux(U, self.lat.axis[k])
        return [self.w * U[m] + self.lat.sign[k] * fl[m] / (2 * self.V) for m in range(len(U))]

    # -- population state: f_k^eq(U) = x, eliminated into a polynomial in the normal velocity
    def state(self, k, x):
        """The admissible population state of x for velocity k, or None."""
        s, V, W0 = self.sys, self.V, self.W0
        n, sg = self.lat.axis[k], self.lat.sign[k]
        if isinstance(s, Burgers):
            # x = w u + sg b u^2 / (4V): (sg b / 4V) u^2 + w u - x = 0; convex where w + sg b u / (2V) > 0
            b = mp.mpf(s.b[n])
            cands = mp.polyroots([sg * b / (4 * V), self.w, -x[0]], maxsteps=200, extraprec=80) if b else [x[0] / self.w]
            good = [mp.re(r) for r in cands if abs(mp.im(r)) < mp.mpf(10) ** -30
                    and self.w + sg * b * mp.re(r) / (2 * V) > 0]
            return [good[0]] if len(good) == 1 else None
        x1 = x[0]
        if not x1 > 0:
            return None
        d = s.d
        xt = [x[1 + i] / x1 for i in range(d)]       # tangential velocities: x_t = x_1 u_t
        if isinstance(s, ShallowWater):
            # x_1 = h W / (2V), W = W0 + sg z;  x_n - z x_1 = sg g h^2 / (4V)
            # => 4 V sg (x_n - z x_1) W^2 - 4 g V^2 x_1^2 = 0, a cubic in z
            g = mp.mpf(s.g)
            xn = x[1 + n]
            # (A + B z)(W0 + sg z)^2 - C with A = 4V sg xn, B = -4V sg x1, C = 4 g V^2 x1^2
            A, B, C = 4 * V * sg * xn, -4 * V * sg * x1, 4 * g * V ** 2 * x1 ** 2
            coeffs = [B * sg * sg, A * sg * sg + 2 * B * W0 * sg, 2 * A * W0 * sg + B * W0 ** 2, A * W0 ** 2 - C]
            good = []
            for r in mp.polyroots(coeffs, maxsteps=400, extraprec=120):
                if abs(mp.im(r)) > mp.mpf(10) ** -25:
                    continue
                z = mp.re(r)
                Wp = W0 + sg * z
                if not Wp > 0:
                    continue
                h = 2 * V * x1 / Wp
                if h > 0 and Wp ** 2 > g * h:
                    vel = [z if i == n else xt[i] for i in range(d)]
                    good.append([h] + [h * c for c in vel])
            return good[0] if len(good) == 1 else None
        gm = mp.mpf(s.gamma)
        xn, xE = x[1 + n], x[1 + d]
        ut2 = sum(xt[i] ** 2 for i in range(d) if i != n)
        # p = 2V sg (x_n - z x_1), W = W0 + sg z, rho W = 2 V x_1, and
        # E W + sg z p = 2V x_E with E = p/(gamma-1) + rho (z^2 + |u_t|^2)/2:
        #   p W/(gamma-1) + V x_1 (z^2 + |u_t|^2) + sg z p - 2V x_E = 0, a quadratic in z
        P0, P1 = 2 * V * sg * xn, -2 * V * sg * x1        # p = P0 + P1 z
        c2 = P1 * sg / (gm - 1) + V * x1 + sg * P1
        c1 = (P0 * sg + P1 * W0) / (gm - 1) + sg * P0
        c0 = P0 * W0 / (gm - 1) + V * x1 * ut2 - 2 * V * xE
        good = []
        for r in mp.polyroots([c2, c1, c0], maxsteps=200, extraprec=80):
            if abs(mp.im(r)) > mp.mpf(10) ** -25:
                continue
            z = mp.re(r)
            Wp = W0 + sg * z
            p = P0 + P1 * z
            if not (Wp > 0 and p > 0):
                continue
            rho = 2 * V * x1 / Wp
            if rho > 0 and rho * Wp ** 2 > gm * p:
                vel = [z if i == n else xt[i] for i in range(d)]
                good.append([rho] + [rho * c for c in vel] + [p / (gm - 1) + rho * sum(c * c for c in vel) / 2])
        return good[0] if len(good) == 1 else None

    def s_k(self, k, x):
        """s_k(x) = v(U).x - s_k^*(v(U)) with f_k^eq(U) = x (None outside the domain)."""
        U = self.state(k, x)
        if U is None:
            return None
        vv = self.v(U)
        n = self.lat.axis[k]
        Sstar = sum(a * b for a, b in zip(vv, U)) - self.S(U)
        Gstar = sum(a * b for a, b in zip(self.flux(U, n), vv)) - self.G(U, n)
        return sum(a * b for a, b in zip(vv, x)) - (self.w * Sstar + self.lat.sign[k] * Gstar / (2 * self.V))

    def sigma(self, fe, dd, t):
        tot = mp.mpf(0)
        for k in range(self.lat.q):
            sk = self.s_k(k, [fe[k][m] + t * dd[k][m] for m in range(len(fe[k]))])
            if sk is None:
                return None
            tot += sk
        return tot


def far_inputs(case):
    """The stage inputs of the far-from-equilibrium GPU parity tests (same generators, same seeds)."""
    system, rel = case
    if system in ("euler", "sw2d"):
        lat = Lattice("D2Q4")
        nx, ny = 67, 29
        rng = np.random.default_rng(31)
        if system == "euler":
            sys, V = Euler(1.4, 2), 3.2
            u = W.euler2d(nx, ny=ny, amp=0.1).initial_state()
        else:
            sys, V = ShallowWater(9.81, 2), 8.0
            u = np.stack([1.0 + 0.05 * rng.standard_normal((ny, nx)), 0.05 * rng.standard_normal((ny, nx)),
                          0.05 * rng.standard_normal((ny, nx))])
    else:
        lat = Lattice("D1Q2")
        n = 3001
        rng = np.random.default_rng(32)
        if system == "sw1d":
            sys, V = ShallowWater(9.81, 1), 4.5
            u = np.stack([1.0 + 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n)])[:, None, :]
        else:
            sys, V = Burgers((1.0,)), 2.0
            u = (0.4 + 0.1 * rng.standard_normal(n))[None, None, :]
    feq = equilibrium(lat, sys, V, u)
    f0 = feq + rel * np.abs(feq) * rng.uniform(-1.0, 1.0, feq.shape)
    return lat, sys, V, f0


CASES = [("euler", 0.05), ("euler", 0.15), ("sw2d", 0.05), ("sw2d", 0.15), ("sw2d", 0.3),
         ("sw1d", 0.05), ("sw1d", 0.2), ("burgers1d", 0.05), ("burgers1d", 0.3)]


def bracketed_root(sig, S1, hint):
    """L with Sigma(f^eq - L d) = Sigma(f): H(L) = Sigma(-L) - Sigma(1) is negative near L = 0 and
    positive past the root; a point outside the domain counts as past it.  The oracle's lambda
    only places the first upper end."""
    H = lambda L: None if sig(L) is None else sig(L) - S1
    lo, hi = mp.mpf("0.05"), hint * (1 + mp.mpf("0.05"))
    assert H(lo) < 0
    while True:
        v = H(hi)
        if v is None or v > 0:
            break
        lo, hi = hi, hi * mp.mpf("1.5")
    if v is not None:
        return mp.findroot(H, (lo, hi), solver="anderson")
    for _ in range(120):       # bisection to 2^-120 of the bracket
        mid = (lo + hi) / 2
        v = H(mid)
        if v is None or v > 0:
            hi = mid
        else:
            lo = mid
    return (lo + hi) / 2


def _node(lat, f0, c):
    q, M = f0.shape[:2]
    fc = f0.reshape(q, M, -1)[:, :, c]
    u = fc.sum(axis=0)
    return fc, u


def _mp_split(model, fc):
    """u, f^eq(u) and d = f - f^eq in mpmath from the binary64 populations (the same numbers the oracle sees)."""
    q, M = fc.shape
    fm = [[mp.mpf(float(fc[k, m])) for m in range(M)] for k in range(q)]
    U = [sum(fm[k][m] for k in range(q)) for m in range(M)]
    fe = [model.feq(k, U) for k in range(q)]
    dd = [[fm[k][m] - fe[k][m] for m in range(M)] for k in range(q)]
    return fe, dd


@pytest.mark.parametrize("case", CASES, ids=["%s-%g" % c for c in CASES])
def test_far_from_equilibrium_lambda_and_fallback_against_brute_force(case):
    lat, sys, V, f0 = far_inputs(case)
    g, om, fb = relax_entropic(lat, sys, V, f0, return_info=True)
    om, fb = om.ravel(), fb.ravel()
    model = Model(lat, sys, V)
    q, M = f0.shape[:2]
    flat = f0.reshape(q, M, -1)
    # nodes with a root: the three farthest from omega = 2 and two random ones
    rooted = np.flatnonzero(~fb)
    rng = np.random.default_rng(77)
    far = rooted[np.argsort(-np.abs(om[rooted] - 2.0))[:3]]
    picks = list(far) + list(rng.choice(rooted, size=2, replace=False))
    for c in picks:
        fc = flat[:, :, c]
        fe, dd = _mp_split(model, fc)
        S1 = model.sigma(fe, dd, 1)
        assert S1 is not None
        lam = om[c] - 1.0
        root = bracketed_root(lambda L: model.sigma(fe, dd, -L), S1, mp.mpf(lam))
        dmax = float(np.max(np.abs(fc - equilibrium(lat, sys, V, fc.sum(0)[:, None])[:, :, 0])))
        fmax = float(np.max(np.abs(fc)))
        assert abs(lam - float(root)) * dmax <= 4 * EPS * fmax, (c, lam, float(root))
    # fallback nodes: no admissible root.  Up to three of each kind, in a seeded order:
    # f itself outside the domain, and the domain edge reached before the root
    fall = rng.permutation(np.flatnonzero(fb))
    seen = {"outside": 0, "edge": 0}
    for c in fall:
        if min(seen.values()) >= 3:
            break
        fc = flat[:, :, c]
        fe, dd = _mp_split(model, fc)
        S1 = model.sigma(fe, dd, 1)
        if S1 is None:
            seen["outside"] += 1      # some population of f has no admissible state
            continue
        if seen["edge"] >= 3:
            continue
        seen["edge"] += 1
        # scan L upward to the first point outside the domain, then bisect to its edge
        L, step = mp.mpf(0), mp.mpf("0.02")
        while L < 8 and model.sigma(fe, dd, -(L + step)) is not None:
            L += step
        assert L < 8, "no domain edge found for a fallback node"
        a, b = L, L + step
        for _ in range(60):
            mid = (a + b) / 2
            if model.sigma(fe, dd, -mid) is None:
                b = mid
            else:
                a = mid
        edge_val = model.sigma(fe, dd, -a) - S1
        assert edge_val < 0, (c, float(edge_val))
    if fall.size >= 20:
        assert seen["outside"] >= 1 and seen["edge"] >= 1, seen
