"""Relaxation phase R_omega and the entropy-limited relaxation parameter.

Test infrastructure only (see ``oracle/__init__``).

R_omega (eq. relaxationDiscretizationOmega):
    f_k <- (1 - omega) f_k + omega f_k^eq(u),  u = sum_k f_k (conserved).

Entropy-limited omega (Sec. 4, eq. variableOmegaProblem): at every node find
omega with  Sigma(R_omega f) - Sigma(f) = 0.  With d_k = f_k - f_k^eq and
lambda = omega - 1 the relaxed state is f^eq - lambda d, and because the
equilibrium minimises Sigma under the moment constraint (eq.
entropyDefinitionMinimization),
    Sigma(f^eq + t d) = S(u) + F(t),  F(t) = sum_k B_k(f_k^eq + t d_k),
with B_k the Bregman divergence of s_k at f_k^eq.  The problem becomes
    F(-lambda) = F(1),  lambda > 0,
the form in which the distance from equilibrium is factored out (Sec. 5.1):
F vanishes to second order at t = 0, and F is evaluated from state differences,
never as a difference of O(1) entropies.  F is strictly convex with its minimum
0 at t = 0, so the root is unique.

Readings (the paper is silent):
  * d = 0 (cell at equilibrium): omega = 2, the limit of the root.
  * no root inside the convexity domain, or the current f itself outside it:
    omega = 1 (projection on equilibrium; conserves u, never increases Sigma),
    counted as a fallback.
Root finder: safeguarded Newton with a bisection bracket (the paper uses a
dichotomy for Burgers and a quasi-Newton method for shallow water; any method
that converges to the unique root gives the same omega up to rounding).
"""
import numpy as np

from .systems import bregman_sum, equilibrium

EPS = np.finfo(np.float64).eps


def relax_fixed(lat, sys, V, f, omega):
    """R_omega with a constant omega (omega = 2: the involution R of Sec. 2.1.2)."""
    u = f.sum(axis=0)
    feq = equilibrium(lat, sys, V, u)
    return (1.0 - omega) * f + omega * feq


def entropic_lambda(lat, sys, V, u, feq, d, maxit=200):
    """Solve F(-lambda) = F(1) per cell; return (lambda, fallback mask).

    u, feq, d are (M, n) / (q, M, n) arrays over n cells.
    """
    n = u.shape[1]
    one = np.ones(n)
    F1, _, ok1 = bregman_sum(lat, sys, V, u, feq, d, one)
    lam = np.ones(n)
    at_eq = np.all(d == 0, axis=(0, 1))
    fallback = ~ok1 & ~at_eq
    active = ok1 & ~at_eq & (F1 > 0)
    lo = np.zeros(n)
    hi = np.full(n, np.inf)
    hi_bad = np.zeros(n, bool)  # hi was set by a point outside the domain
    x = np.ones(n)
    dmax = np.max(np.abs(d), axis=(0, 1))
    fmax = np.maximum(np.max(np.abs(feq), axis=(0, 1)), np.max(np.abs(feq + d), axis=(0, 1)))
    for _ in range(maxit):
        if not active.any():
            break
        idx = np.flatnonzero(active)
        xa = x[idx]
        Fx, dFx, okx = bregman_sum(lat, sys, V, u[:, idx], feq[:, :, idx], d[:, :, idx], -xa)
        H = Fx - F1[idx]           # H(lambda) = F(-lambda) - F(1), increasing in lambda
        dH = -dFx
        above = ~okx | (H > 0)
        exact = okx & (H == 0)
        hi_i = np.where(above, np.minimum(hi[idx], xa), hi[idx])
        hi_bad[idx] = np.where(above & (xa <= hi[idx]), ~okx, hi_bad[idx])
        lo_i = np.where(~above, np.maximum(lo[idx], xa), lo[idx])
        hi[idx], lo[idx] = hi_i, lo_i
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = xa - H / dH
        newton_ok = okx & np.isfinite(xn) & (xn > lo_i) & (xn < hi_i)
        xb = np.where(np.isinf(hi_i), 2.0 * xa, 0.5 * (lo_i + hi_i))
        xnew = np.where(exact, xa, np.where(newton_ok, xn, xb))
        # lambda only enters through f^eq - lambda d: stop once a step no longer
        # changes the relaxed populations by more than rounding
        small_step = newton_ok & (np.abs(xnew - xa) * dmax[idx] <= 2.0 * EPS * fmax[idx])
        collapsed = np.isfinite(hi_i) & ((hi_i - lo_i) * dmax[idx] <= 2.0 * EPS * fmax[idx])
        done = exact | small_step | collapsed
        x[idx] = np.where(collapsed & ~exact & ~small_step, np.where(hi_bad[idx], lo_i, hi_i), xnew)
        # a bracket that collapsed against the edge of the domain has no root inside it
        nores = collapsed & ~exact & ~small_step & hi_bad[idx]
        fallback[idx[nores]] = True
        active[idx[done]] = False
    if active.any():
        raise RuntimeError("entropic omega: root finder did not converge in %d iterations" % maxit)
    lam = np.where(~ok1 | at_eq, lam, x)
    lam = np.where(fallback, 0.0, lam)
    return lam, fallback


def relax_entropic(lat, sys, V, f, return_info=False):
    """R_omega(f) f with omega(f) from eq. variableOmegaProblem, per node."""
    q, M = f.shape[:2]
    shp = f.shape[2:]
    fc = f.reshape(q, M, -1)
    u = fc.sum(axis=0)
    feq = equilibrium(lat, sys, V, u)
    d = fc - feq
    lam, fb = entropic_lambda(lat, sys, V, u, feq, d)
    out = (feq - lam * d).reshape(f.shape)
    if return_info:
        return out, (lam + 1.0).reshape(shp), fb.reshape(shp)
    return out
