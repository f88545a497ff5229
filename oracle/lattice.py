"""Velocity sets, transport phase and time step.

Test infrastructure only (see ``oracle/__init__``).

State layout used throughout the oracle: ``f[k, m, y, x]`` (float64), ``k`` the
discrete velocity, ``m`` the conserved component, ``x`` fastest; 1D problems
have ``ny == 1``.  Velocity order follows Sec. 1.2.1 (``+``, ``-``) and
Sec. 1.2.2 (``+x``, ``+y``, ``-x``, ``-y``).
"""
import numpy as np


class Lattice:
    """DdQq velocity set with V_k in V * Z^d (Sec. 1.2.1, Sec. 1.2.2)."""

    def __init__(self, name):
        if name == "D1Q2":
            self.d, self.q = 1, 2
            self.c = np.array([[1], [-1]])
        elif name == "D2Q4":
            self.d, self.q = 2, 4
            self.c = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]])
        else:
            raise ValueError(name)
        self.name = name
        # f_k^eq = u / q + (V_k / V) . phi / (2V): weight of u in every equilibrium
        self.w = 1.0 / self.q
        # every velocity here lies on one axis; keep its axis and sign
        self.axis = [int(np.flatnonzero(ck)[0]) for ck in self.c]
        self.sign = [int(ck[a]) for ck, a in zip(self.c, self.axis)]


def transport(lat, f, s):
    """T(s): pull shift by s cells along each velocity, periodic (eq. transportPhase).

    f_k(x) <- f_k(x - s c_k dx), with c_k = V_k / V in Z^d; a negative s moves the
    populations against their velocity (Sec. 2.1.3, negative time steps).  This is
    exactly numpy.roll: roll(a, r)[i] == a[i - r].
    """
    out = np.empty_like(f)
    for k in range(lat.q):
        ck = lat.c[k]
        g = f[k]
        # axis -1 is x, axis -2 is y (arrays are [m, y, x])
        g = np.roll(g, s * int(ck[0]), axis=-1)
        if lat.d == 2:
            g = np.roll(g, s * int(ck[1]), axis=-2)
        out[k] = g
    return out


def time_step(dx, V, kappa=1):
    """Delta t = 24 kappa dx / V: the shortest transport moves kappa cells (Sec. 2.3)."""
    return 24.0 * kappa * dx / V


def steps_for_time(T, dt):
    """Number of composed steps to reach T.

    The paper does not say how a final time that is not a multiple of Delta t is
    handled.  Reading: n = floor(T / Delta t) evaluated in FP64, and the solution is
    compared at t_n = n Delta t.  This reproduces Table 1 (N = 500: 2 steps) and
    Table 6 (N = 20: 9 steps).
    """
    return int(np.floor(T / dt))


def grid(n):
    """Nodes x_j = j dx, j = 0..n-1, dx = 1/n on the periodic unit interval.

    Silent in the paper; this node set reproduces Table 2's Err-Estim when the
    N run is compared with every other node of the 2N run.
    """
    dx = 1.0 / n
    return np.arange(n) * dx, dx
