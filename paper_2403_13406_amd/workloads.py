"""Seeded synthetic workloads (initial conserved states and problem settings).

This module draws random numbers and evaluates smooth initial fields only; it
holds none of the scheme's arithmetic, so both the HIP path and the CPU oracle
may be fed from it.  The shapes follow the paper's smooth periodic tests
(Sec. 3: sine data on [0,1] / [0,1]^2 at equilibrium); no dataset is involved.

Workloads
---------
burgers1d   1D Burgers, D1Q2, N = 1024, V = 2, T = 0.2 (17 composed steps);
            u0 = 0.5 + 0.25 sin 2 pi x + sum_{k=1..4} a_k sin(2 pi k x + phi_k),
            a_k ~ U(0, 0.02), phi_k ~ U(0, 2 pi).
sw1d        1D shallow water, D1Q2^2, N = 2^20, g = 9.81, V = 4.5, 4000 steps;
            h0 = 1 + 0.1 sin 2 pi x + sum_{k=1..4} a_k sin(...), a_k ~ U(0, 0.01), u0 = 0.
euler2d     2D Euler, D2Q4^4, 4096^2, gamma = 1.4, V = 3.2, 500 steps;
            rho = 1 + P_rho, u = P_u, v = P_v, p = 1, each P a sum of cosines over
            1 <= |k|_inf <= 8 with amplitude xi_k |k|^-3 (xi_k ~ U(0,1)) and random
            phases, rescaled to max |P| = 0.05.
sw2d_batch  512 instances of 2D shallow water, D2Q4^3; for instance i, rng(1000+i)
            draws n_i in {64,128,256,512,1024} and a step count in [100, 1000];
            g = 9.81, V = 8, h = 1 + 0.05 P_h, hu = 0.02 P_u, hv = 0.02 P_v, |k| <= 4.
euler2d_adjoint  2D Euler at 1024^2, V = 3.2, amplitude 0.005, 2000 steps; target
            state from seed 1; finite-difference directions from seed 2.
riemann2d   2D Euler four-quadrant Riemann problem (Sec. 6.3 setting: gamma = 1.4,
            V = 6.21, T = 0.25, 1024^2 or 2048^2), constant states (rho, u, v, p)
            split at x = 1/2, y = 1/2:  x>1/2,y>1/2: (1, 0, 0, 1);  x<1/2,y>1/2:
            (0.6, 0.3, 0, 0.5);  x<1/2,y<1/2: (1, 0.3, 0.3, 1);  x>1/2,y<1/2:
            (0.6, 0, 0.3, 0.5).  Our own states, symmetric about the diagonal, with
            flows converging on the upper-right quadrant; they stand in for the
            configuration of the cited Riemann-problem study, which is not
            reproduced.  The domain is periodic (a 2x2 checkerboard of the states).
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    lattice: str
    system: str
    nx: int
    ny: int
    V: float
    param: tuple
    nsteps: int
    seed: int = 0
    relax: str = "entropic"
    extra: dict = field(default_factory=dict)

    @property
    def dx(self):
        return 1.0 / self.nx

    @property
    def cells(self):
        return self.nx * self.ny

    def initial_state(self):
        return initial_state(self)


def _sines_1d(n, rng, kmax, amax):
    x = np.arange(n) / n
    a = rng.uniform(0.0, amax, size=kmax)
    ph = rng.uniform(0.0, 2 * np.pi, size=kmax)
    out = np.zeros(n)
    for k in range(1, kmax + 1):
        out += a[k - 1] * np.sin(2 * np.pi * k * x + ph[k - 1])
    return x, out


def spectral_field_2d(nx, ny, rng, kmax, amp):
    """sum over 1 <= |k|_inf <= kmax of xi_k |k|^-3 cos(2 pi k.x + phi_k), rescaled to max |P| = amp."""
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if max(abs(kx), abs(ky)) >= 1]
    xi = rng.uniform(0.0, 1.0, size=len(ks))
    ph = rng.uniform(0.0, 2 * np.pi, size=len(ks))
    C = np.zeros((2 * kmax + 1, 2 * kmax + 1), complex)   # [ky, kx]
    for (kx, ky), a, p in zip(ks, xi, ph):
        C[ky + kmax, kx + kmax] += a * np.hypot(kx, ky) ** -3 * np.exp(1j * p)
    kk = np.arange(-kmax, kmax + 1)
    Ex = np.exp(2j * np.pi * np.outer(kk, np.arange(nx) / nx))   # [kx, x]
    Ey = np.exp(2j * np.pi * np.outer(np.arange(ny) / ny, kk))   # [y, ky]
    P = (Ey @ C @ Ex).real
    return amp * P / np.max(np.abs(P))


def initial_state(w):
    """Conserved variables u0 as a float64 array (M, ny, nx)."""
    rng = np.random.default_rng(w.seed)
    if w.name.startswith("burgers1d"):
        x, pert = _sines_1d(w.nx, rng, 4, 0.02)
        u = 0.5 + 0.25 * np.sin(2 * np.pi * x) + pert
        return u[None, None, :].copy()
    if w.name.startswith("sw1d"):
        x, pert = _sines_1d(w.nx, rng, 4, 0.01)
        h = 1.0 + 0.1 * np.sin(2 * np.pi * x) + pert
        return np.stack([h, np.zeros_like(h)])[:, None, :].copy()
    if w.name.startswith("euler2d"):
        amp = w.extra.get("amp", 0.05)
        gamma = w.param[0]
        Pr = spectral_field_2d(w.nx, w.ny, rng, 8, amp)
        Pu = spectral_field_2d(w.nx, w.ny, rng, 8, amp)
        Pv = spectral_field_2d(w.nx, w.ny, rng, 8, amp)
        rho = 1.0 + Pr
        p = np.ones_like(rho)
        E = 0.5 * rho * (Pu ** 2 + Pv ** 2) + p / (gamma - 1.0)
        return np.stack([rho, rho * Pu, rho * Pv, E])
    if w.name.startswith("riemann2d"):
        gamma = w.param[0]
        x = np.arange(w.nx) / w.nx
        y = np.arange(w.ny) / w.ny
        right = (x >= 0.5)[None, :]
        top = (y >= 0.5)[:, None]
        prim = {(True, True): (1.0, 0.0, 0.0, 1.0), (False, True): (0.6, 0.3, 0.0, 0.5),
                (False, False): (1.0, 0.3, 0.3, 1.0), (True, False): (0.6, 0.0, 0.3, 0.5)}
        rho, u, v, p = (np.zeros((w.ny, w.nx)) for _ in range(4))
        for (r, t), (a, b, c, d) in prim.items():
            mask = np.logical_and(right == r, top == t)
            rho[mask], u[mask], v[mask], p[mask] = a, b, c, d
        E = 0.5 * rho * (u ** 2 + v ** 2) + p / (gamma - 1.0)
        return np.stack([rho, rho * u, rho * v, E])
    if w.name.startswith("sw2d"):
        Ph = spectral_field_2d(w.nx, w.ny, rng, 4, 1.0)
        Pu = spectral_field_2d(w.nx, w.ny, rng, 4, 1.0)
        Pv = spectral_field_2d(w.nx, w.ny, rng, 4, 1.0)
        h = 1.0 + 0.05 * Ph
        return np.stack([h, 0.02 * Pu, 0.02 * Pv])
    raise ValueError(w.name)


def burgers1d(n=1024, seed=0):
    return Workload("burgers1d", "D1Q2", "burgers", n, 1, 2.0, (1.0,), 17, seed)


def sw1d(n=1 << 20, seed=0, nsteps=4000):
    return Workload("sw1d", "D1Q2", "shallow_water", n, 1, 4.5, (9.81,), nsteps, seed)


def euler2d(n=4096, ny=None, seed=0, nsteps=500, amp=0.05):
    return Workload("euler2d", "D2Q4", "euler", n, ny or n, 3.2, (1.4,), nsteps, seed, extra={"amp": amp})


def euler2d_adjoint(n=1024, seed=0, nsteps=2000):
    return Workload("euler2d_adjoint", "D2Q4", "euler", n, n, 3.2, (1.4,), nsteps, seed,
                    extra={"amp": 0.005, "ckpt_every": 50, "target_seed": 1, "fd_seed": 2, "fd_dirs": 32})


# schemes of the Sec. 6.3 comparison: (A) standard LB with omega = 1.93, (B) the
# projected basic brick, (C) the fourth-order scheme with omega = 2 and
# projections after every brick (Scheme III)
RIEMANN_SCHEMES = {"A": dict(scheme=5, relax="fixed", omega=1.93),
                   "B": dict(scheme=6, relax="fixed", omega=2.0),
                   "C": dict(scheme=3, relax="fixed", omega=2.0)}


def riemann2d(n=1024, T=0.25):
    return Workload("riemann2d", "D2Q4", "euler", n, n, 6.21, (1.4,), 0, 0, relax="fixed", extra={"T": T})


def sw2d_instance(i):
    """Instance i of the batched ensemble (its own seed 1000 + i)."""
    rng = np.random.default_rng(1000 + i)
    n = int(rng.choice([64, 128, 256, 512, 1024]))
    steps = int(rng.integers(100, 1001))
    return Workload("sw2d_%d" % i, "D2Q4", "shallow_water", n, n, 8.0, (9.81,), steps, 1000 + i)


def sw2d_batch(count=512):
    return [sw2d_instance(i) for i in range(count)]
