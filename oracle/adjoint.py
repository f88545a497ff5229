"""Plain adjoint (reverse-mode derivative) of the relaxation stage and of the time loop.

Test infrastructure only (see ``oracle/__init__``).

The paper has no adjoint; this is the derivative of its scheme.  One relaxation
(eq. relaxationDiscretizationOmega) maps the stage input h to
    g_k = (1 - omega) h_k + omega f_k^eq(u),   u = sum_k h_k,
so, for a cotangent gbar of g,
    hbar_j = (1 - omega) gbar_j + omega sum_k J_k^T gbar_k
             + grad_{h_j} omega * sum_k (f_k^eq - h_k) . gbar_k,
J_k = d f_k^eq / du.  With the entropy-limited omega (eq. variableOmegaProblem),
Phi(omega, h) = Sigma(g) - Sigma(h) = 0 defines omega(h) and
    grad_{h_j} omega = -(d Phi / d h_j) / (d Phi / d omega),
    d Phi / d omega = -F'(-lambda),
    d Phi / d h_j  = (1 - omega) dv_j(-lambda) + omega sum_k J_k^T dv_k(-lambda) - dv_j(1),
with dv_k(t) = v(U_k(t)) - v(u) the entropy-variable offset of the population
state of f_k^eq + t d_k (the constant v(u) drops out because sum_k J_k = I and
sum_k d_k = 0).  Every factor is a difference, so nothing O(1) cancels.
Fixed omega, and nodes that fell back to omega = 1, use the first two terms.

J_k^T y is obtained by complex-step differentiation of the oracle's equilibrium
(exact to rounding for these analytic fluxes), not from hand-written Jacobians.
The adjoint of the transport T(s) is T(-s).
"""
import numpy as np

from .lattice import transport
from .relaxation import entropic_lambda
from .systems import equilibrium

_CSTEP = 1e-30


def eq_jacobian_T(lat, sys, V, u, y):
    """sum_k J_k(u)^T y_k per node; u (M, n), y (q, M, n) -> (M, n)."""
    M = u.shape[0]
    out = np.zeros_like(u)
    for c in range(M):
        up = u.astype(complex)
        up[c] = up[c] + 1j * _CSTEP
        dfeq = equilibrium(lat, sys, V, up).imag / _CSTEP     # d f^eq_{k,m} / d u_c
        out[c] = np.sum(dfeq * y, axis=(0, 1))
    return out


def _dv_all(lat, sys, V, u, feq, d, t):
    dvs = []
    for k in range(lat.q):
        _, dv, _ = sys.bregman(lat, V, k, u, feq[k], t * d[k])
        dvs.append(dv)
    return np.array(dvs)


def relax_adjoint(lat, sys, V, h, gbar, mode="entropic", omega=2.0):
    """hbar for one relaxation pass with input h (logical layout (q, M, ny, nx))."""
    q, M = h.shape[:2]
    shp = h.shape
    hc = h.reshape(q, M, -1)
    gb = gbar.reshape(q, M, -1)
    u = hc.sum(axis=0)
    feq = equilibrium(lat, sys, V, u)
    d = hc - feq
    n = u.shape[1]
    if mode == "fixed":
        om = np.full(n, float(omega))
        fallback = np.ones(n, bool)
        lam = om - 1.0
    else:
        lam, fallback = entropic_lambda(lat, sys, V, u, feq, d)
        om = lam + 1.0
    JTg = eq_jacobian_T(lat, sys, V, u, gb)
    hbar = (1.0 - om) * gb + om * JTg[None]
    if mode != "fixed":
        at_eq = np.all(d == 0, axis=(0, 1))
        use = ~fallback & ~at_eq
        if use.any():
            dvm = _dv_all(lat, sys, V, u, feq, d, -lam)          # dv_k(-lambda)
            dv1 = _dv_all(lat, sys, V, u, feq, d, np.ones(n))    # dv_k(1)
            Fp = np.sum(dvm * d, axis=(0, 1))                    # F'(-lambda)
            JTdv = eq_jacobian_T(lat, sys, V, u, dvm)
            dPhi_dh = (1.0 - om) * dvm + om * JTdv[None] - dv1
            c = -np.sum(d * gb, axis=(0, 1))                     # sum_k (f^eq_k - h_k) . gbar_k
            with np.errstate(divide="ignore", invalid="ignore"):
                term = dPhi_dh * (c / Fp)[None, None]
            hbar = hbar + np.where(use[None, None], term, 0.0)
    return hbar.reshape(shp)


def step_operations(kappa=1, scheme=1):
    """The composed step as a flat list: ('T', cells) or ('R',) or ('P',) (eq. splittingToUse)."""
    ops = []
    a, b = 4 * kappa, -8 * kappa
    for c in [a] * 4 + [b] + [a] * 4:
        ops += [("T", c // 4), ("R",), ("T", c // 2), ("R",), ("T", c // 4)]
        if scheme == 3:
            ops.append(("P",))
    if scheme == 2:
        ops.append(("P",))
    return ops


def forward_with_tape(relax, f, nsteps, kappa=1, scheme=1):
    """Run n steps and keep every relaxation input (the tape), plain and memory-hungry."""
    from .relaxation import relax_fixed
    tape = []
    ops = step_operations(kappa, scheme) * nsteps
    for op in ops:
        if op[0] == "T":
            f = transport(relax.lat, f, op[1])
        elif op[0] == "R":
            tape.append(f)
            f = relax(f)
        else:
            tape.append(f)
            f = relax_fixed(relax.lat, relax.sys, relax.V, f, 1.0)
    return f, tape, ops


def adjoint_run(relax, f0, nsteps, fbar_T, kappa=1, scheme=1):
    """fbar(0) from fbar(T) through n composed steps (reverse sweep over the tape)."""
    _, tape, ops = forward_with_tape(relax, f0, nsteps, kappa, scheme)
    fbar = fbar_T
    for op in reversed(ops):
        if op[0] == "T":
            fbar = transport(relax.lat, fbar, -op[1])
        elif op[0] == "R":
            h = tape.pop()
            fbar = relax_adjoint(relax.lat, relax.sys, relax.V, h, fbar, relax.mode, relax.omega)
        else:
            h = tape.pop()
            fbar = relax_adjoint(relax.lat, relax.sys, relax.V, h, fbar, "fixed", 1.0)
    return fbar


def init_adjoint(lat, sys, V, u0, fbar0):
    """ubar_0 = sum_k J_k(u0)^T fbar_k(0) for f(0) = f^eq(u0) (Sec. 3.1 initialisation)."""
    shp = u0.shape
    M = shp[0]
    q = fbar0.shape[0]
    return eq_jacobian_T(lat, sys, V, u0.reshape(M, -1), fbar0.reshape(q, M, -1)).reshape(shp)


def misfit_gradient(relax, u0, u_target, nsteps, kappa=1, scheme=1):
    """L = 1/2 sum_x sum_m (U_m(T) - U_target,m)^2 with U(T) = sum_k f_k(T); returns (L, dL/du0)."""
    lat, sys, V = relax.lat, relax.sys, relax.V
    f0 = equilibrium(lat, sys, V, u0)
    fT, tape, ops = forward_with_tape(relax, f0, nsteps, kappa, scheme)
    r = fT.sum(axis=0) - u_target
    L = 0.5 * float(np.sum(r * r))
    fbar = np.broadcast_to(r[None], fT.shape).copy()       # adjoint of U = sum_k f_k
    for op in reversed(ops):
        if op[0] == "T":
            fbar = transport(lat, fbar, -op[1])
        elif op[0] == "R":
            fbar = relax_adjoint(lat, sys, V, tape.pop(), fbar, relax.mode, relax.omega)
        else:
            fbar = relax_adjoint(lat, sys, V, tape.pop(), fbar, "fixed", 1.0)
    return L, init_adjoint(lat, sys, V, u0, fbar)
