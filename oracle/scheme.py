"""Time-symmetric basic brick, rational composition and the time loop.

Test infrastructure only (see ``oracle/__init__``).

Transport lengths are counted in cells.  With Delta t = 24 kappa dx / V
(Sec. 2.3), the transport T(tau) moves every population by V tau / dx =
24 kappa tau / Delta t cells; kappa = 1 throughout the paper.

basic brick (eq. basicBrickSplitting):
    psi(tau) = T(tau/4) R T(tau/2) R T(tau/4)
composition (eq. splittingToUse):
    Phi(Delta t) = psi(Delta t/6)^4 psi(-Delta t/3) psi(Delta t/6)^4
so psi(Delta t/6) moves 1, 2, 1 cells and psi(-Delta t/3) moves -2, -4, -2.
Both operators are palindromes, so the order of application inside a product
is immaterial.  The oracle applies the bricks literally, one transport at a
time, with no merging of consecutive shifts.

Projections (Sec. 6.1): Scheme II applies R_1 after Phi; Scheme III applies
R_1 after every psi.  The standard second-order lattice Boltzmann scheme is
R T(Delta t) (Sec. 2.1.3); the fair comparison of Sec. 3.1 advances Delta t
with (R T(Delta t / 24))^24.
"""
from .lattice import transport
from .relaxation import relax_entropic, relax_fixed


class Relaxer:
    """R applied inside the bricks: omega fixed (2 in the paper) or entropy-limited."""

    def __init__(self, lat, sys, V, mode="fixed", omega=2.0):
        self.lat, self.sys, self.V = lat, sys, V
        self.mode, self.omega = mode, omega

    def __call__(self, f):
        if self.mode == "fixed":
            return relax_fixed(self.lat, self.sys, self.V, f, self.omega)
        return relax_entropic(self.lat, self.sys, self.V, f)

    def project(self, f):
        """R_1: projection on the equilibrium (Sec. 6.1)."""
        return relax_fixed(self.lat, self.sys, self.V, f, 1.0)


def brick(relax, f, cells):
    """psi(tau) with V tau / dx = 4 * cells / ... : shifts cells/4, cells/2, cells/4.

    ``cells`` is the total movement of the brick (4 for psi(Delta t / 6) with
    kappa = 1, -8 for psi(-Delta t / 3)).
    """
    assert cells % 4 == 0
    lat = relax.lat
    f = transport(lat, f, cells // 4)
    f = relax(f)
    f = transport(lat, f, cells // 2)
    f = relax(f)
    f = transport(lat, f, cells // 4)
    return f


def composed_step(relax, f, kappa=1, scheme=1):
    """One step of Phi(Delta t), eq. splittingToUse (Scheme I); Schemes II/III of Sec. 6.1."""
    a, b = 4 * kappa, -8 * kappa   # psi(Delta t / 6) and psi(-Delta t / 3), in cells
    for c in [a] * 4 + [b] + [a] * 4:
        f = brick(relax, f, c)
        if scheme == 3:
            f = relax.project(f)
    if scheme == 2:
        f = relax.project(f)
    return f


def standard_lb_step(relax, f, kappa=1):
    """(R T(Delta t / 24))^24: the second-order comparator of Sec. 3.1 (Figure fairComparison)."""
    for _ in range(24):
        f = transport(relax.lat, f, kappa)
        f = relax(f)
    return f


def run(relax, f, nsteps, kappa=1, scheme=1, callback=None):
    """n composed steps; ``callback(i, f)`` after each one (diagnostics)."""
    for i in range(nsteps):
        f = composed_step(relax, f, kappa, scheme)
        if callback is not None:
            callback(i, f)
    return f


def moments(f):
    """u = sum_k f_k (Sec. 1.2); meaningful at step boundaries (Sec. 2.3, cost remark)."""
    return f.sum(axis=0)


def scheme_A_step(relax, f, kappa=1):
    """Scheme (A) of Sec. 6.3: R T(dt), dt = kappa dx / V (omega chosen by the caller)."""
    return relax(transport(relax.lat, f, kappa))


def scheme_B_step(relax, f, kappa=1):
    """Scheme (B) of Sec. 6.3: R_1 T(dt/4) R T(dt/2) R T(dt/4), dt = 4 kappa dx / V."""
    f = relax(transport(relax.lat, f, kappa))
    f = relax(transport(relax.lat, f, 2 * kappa))
    return relax.project(transport(relax.lat, f, kappa))
