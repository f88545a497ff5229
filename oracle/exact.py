"""Exact solutions and error norms of the convergence experiments (Sec. 3, Sec. 5, Sec. 6).

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np


def l2_error(a, b, dx, d=1):
    """sqrt(dx^d sum |a - b|^2) (the L2 norm of Tables 1, 4, 5, 6)."""
    return float(np.sqrt(dx ** d * np.sum((np.asarray(a) - np.asarray(b)) ** 2)))


def err_estim(coarse, fine, dx, d=1):
    """Err-Estim of Sec. 3.2 / 3.3: coarse run vs every other node of the 2N run."""
    if d == 1:
        f2 = fine[..., ::2]
    else:
        f2 = fine[..., ::2, ::2]
    return l2_error(coarse, f2, dx, d)


def burgers_exact(u0, x, t, iters=100):
    """Entropy solution of u_t + (u^2/2)_x = 0 before the shock: u = u0(xi), xi + u0(xi) t = x.

    Newton on the characteristic foot xi (smooth data, t below the breaking time).
    ``u0`` is a callable with derivative ``u0.d``.
    """
    xi = np.array(x, dtype=np.float64)
    for _ in range(iters):
        r = xi + u0(xi) * t - x
        dr = 1.0 + u0.d(xi) * t
        step = r / dr
        xi = xi - step
        if np.max(np.abs(step)) < 1e-16:
            break
    return u0(xi)


class SinData:
    """u0(x) = c + A sin(2 pi x) + sum_k a_k sin(2 pi k x + phi_k), with its derivative."""

    def __init__(self, c=0.0, A=1.0, modes=()):
        self.c, self.A, self.modes = c, A, tuple(modes)

    def __call__(self, x):
        y = self.c + self.A * np.sin(2 * np.pi * x)
        for k, a, ph in self.modes:
            y = y + a * np.sin(2 * np.pi * k * x + ph)
        return y

    def d(self, x):
        y = 2 * np.pi * self.A * np.cos(2 * np.pi * x)
        for k, a, ph in self.modes:
            y = y + 2 * np.pi * k * a * np.cos(2 * np.pi * k * x + ph)
        return y
