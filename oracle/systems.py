"""Target systems, equilibria, kinetic entropies and population states.

Test infrastructure only (see ``oracle/__init__``).

Sec. 1.1: u_t + sum_j d_j phi^j(u) = 0 with a convex entropy S.
Sec. 1.2: discrete-velocity BGK system; equilibria fixed by the moment
constraints (eq. constraintsKinetic):
    D1Q2:  f_+-^eq = u/2 +- phi(u) / (2V)                      (Sec. 1.2.1)
    D2Q4:  f_+-x/y^eq = u/4 +- phi_x/y(u) / (2V)                (Sec. 1.2.2)
i.e. f_k^eq = w u + sigma_k phi^{n_k}(u) / (2V), w = 1/q, with n_k the axis of
V_k and sigma_k its sign.

Kinetic entropies (Sec. 1.2, eq. entropyDefinitionMinimization and
eq. transformationEntropyFlux).  The dual kinetic entropies are
    s_k^*(p) = w S^*(p) + sigma_k G^{n_k,*}(p) / (2V),
whose gradient is f_k^eq(u(p)); they reproduce the paper's Examples:
    linear transport  s_+-^* = (1 +- a/V) p^2 / 4
    Burgers           s_+-^* = p^2/4 +- p^3 / (12 V)
    shallow water     s_+-^* = (V +- p_2)(2 p_1 + p_2^2)^2 / (16 g V)
                             = g h^2 (V +- u) / (4V) in state variables.
For the Euler system (Sec. 6.3; the paper gives no kinetic entropy for it) the
entropy is S = -rho s / (gamma - 1), s = ln(p rho^-gamma); then S^* = rho and
G^{x,*} = rho u, so s_k^* is the mass component of f_k^eq.

Population state.  A population value x is the equilibrium of exactly one state
U_k on the convex branch ("population state"): f_k^eq(U_k) = x.  Then
s_k(x) = v(U_k).x - s_k^*(v(U_k)) with v = grad S.  The Bregman divergence
    B_k(x) = s_k(x) - s_k(f_k^eq(u)) - v(u).(x - f_k^eq(u))
is written below in closed form as a quadratic-type expression of the state
differences U_k - u, which keeps it accurate when x is close to equilibrium
(the paper's "factorise the distance from equilibrium", Sec. 5.1).  The
differences themselves are solved from the increment e = x - f_k^eq(u): the
equation f_k^eq(u + dU) - f_k^eq(u) = e has its O(1) part cancelled exactly, so
dU carries a relative (not absolute) rounding error; the plain inversion
(population_state) picks the branch and is pinned against numpy.roots.
The closed forms are pinned against 40-digit brute force in the tests.
"""
import numpy as np


def equilibrium(lat, sys, V, u):
    """f_k^eq(u) = w u + sigma_k phi^{n_k}(u) / (2V), shape (q, M, ...)."""
    fl = [sys.flux(u, j) for j in range(lat.d)]
    feq = np.empty((lat.q,) + u.shape, dtype=np.result_type(u, np.float64))
    for k in range(lat.q):
        feq[k] = lat.w * u + lat.sign[k] * fl[lat.axis[k]] / (2.0 * V)
    return feq


def _phi_log(z):
    """phi(z) = z - 1 - ln z >= 0 (convex, zero at z = 1)."""
    return z - 1.0 - np.log(z)


class Advection:
    """Linear transport phi^j = a_j u, S = u^2/2 (Example "Linear transport")."""

    name = "advection"
    M = 1

    def __init__(self, a):
        self.a = tuple(float(x) for x in a)

    def flux(self, u, j):
        return self.a[j] * u

    def macro_entropy(self, u):
        return 0.5 * u[0] ** 2

    def entropy_variable(self, u):
        return u.copy()

    def _wk(self, lat, V, k):
        return lat.w + lat.sign[k] * self.a[lat.axis[k]] / (2.0 * V)

    def bregman(self, lat, V, k, u, feqk, e):
        """s_k(x) = x^2 / (2 w_k), w_k = w + sigma a_n / (2V): w_k dU = e, B = w_k dU^2 / 2."""
        wk = self._wk(lat, V, k)
        with np.errstate(divide="ignore", invalid="ignore"):
            dU = e[0] / wk
        B = 0.5 * wk * dU ** 2
        valid = np.full(dU.shape, wk > 0)
        return B, dU[None], valid

    def admissible(self, u):
        return np.ones(u.shape[1:], bool)

    def subcharacteristic(self, lat, V, u):
        return np.full(u.shape[1:], all(self._wk(lat, V, k) > 0 for k in range(lat.q)))


class Burgers:
    """phi^j = b_j u^2 / 2, S = u^2 / 2 (Example "Burgers' equation"; 2D: Sec. 3.3)."""

    name = "burgers"
    M = 1

    def __init__(self, b=(1.0,)):
        self.b = tuple(float(x) for x in b)

    def flux(self, u, j):
        return 0.5 * self.b[j] * u ** 2

    def macro_entropy(self, u):
        return 0.5 * u[0] ** 2

    def entropy_variable(self, u):
        return u.copy()

    def population_state(self, lat, V, k, x):
        """Solve w U + beta U^2 / (4V) = x, beta = sigma b_n, on the convex branch.

        1D: U = +-V (sqrt(1 +- 4x/V) - 1), the inverse used in the Burgers example.
        The convex branch needs w^2 + beta x / V > 0.
        """
        beta = lat.sign[k] * self.b[lat.axis[k]]
        disc = lat.w ** 2 + beta * x / V
        valid = disc > 0
        U = 2.0 * x / (lat.w + np.sqrt(np.where(valid, disc, 1.0)))
        return U, valid

    def bregman(self, lat, V, k, u, feqk, e):
        """B_k = dU^2 [w/2 + beta (3u + 2 dU) / (12V)], dU = U_k - u (Taylor of the cubic s_k^*).

        Increment form: f_k^eq(u + dU) - f_k^eq(u) = e reads (beta/4V) dU^2 + c1 dU = e,
        c1 = w + beta u / (2V), solved as dU = 2e / (c1 + sqrt(c1^2 + beta e / V)); the
        convex branch needs c1 > 0 (sub-characteristic) and a positive discriminant.
        """
        beta = lat.sign[k] * self.b[lat.axis[k]]
        c1 = lat.w + beta * u[0] / (2.0 * V)
        disc = c1 ** 2 + beta * e[0] / V
        valid = (c1 > 0) & (disc > 0)
        dU = 2.0 * e[0] / (c1 + np.sqrt(np.where(valid, disc, c1 ** 2)))
        B = dU ** 2 * (0.5 * lat.w + beta * (3.0 * u[0] + 2.0 * dU) / (12.0 * V))
        return B, dU[None], valid

    def admissible(self, u):
        return np.ones(u.shape[1:], bool)

    def subcharacteristic(self, lat, V, u):
        ok = np.ones(u.shape[1:], bool)
        for k in range(lat.q):
            beta = lat.sign[k] * self.b[lat.axis[k]]
            ok &= lat.w + beta * u[0] / (2.0 * V) > 0
        return ok


class ShallowWater:
    """u = (h, h u_1..u_d), phi^j = (h u_j, h u_j u + g h^2 e_j / 2) (Example "Shallow water").

    S = h |u|^2 / 2 + g h^2 / 2, v = (g h - |u|^2/2, u).  For population k with
    axis n and sign sigma, W = 2wV + sigma u_n; then
        f^eq_1 = h W / (2V),  f^eq_n = f^eq_1 u_n + sigma g h^2 / (4V),
        f^eq_t = f^eq_1 u_t (tangential),   s_k^* = g h^2 W / (4V).
    """

    name = "shallow_water"

    def __init__(self, g, d=1):
        self.g = float(g)
        self.d = d
        self.M = d + 1

    def flux(self, u, j):
        h = u[0]
        vel = u[1:] / h
        out = np.empty_like(u)
        out[0] = u[1 + j]
        out[1:] = u[1 + j] * vel
        out[1 + j] += 0.5 * self.g * h ** 2
        return out

    def macro_entropy(self, u):
        h = u[0]
        return 0.5 * np.sum(u[1:] ** 2, axis=0) / h + 0.5 * self.g * h ** 2

    def entropy_variable(self, u):
        h = u[0]
        vel = u[1:] / h
        return np.concatenate([(self.g * h - 0.5 * np.sum(vel ** 2, axis=0))[None], vel])

    def population_state(self, lat, V, k, x):
        """Invert f_k^eq(U) = x.

        u_t = x_t / x_1; the normal velocity z solves the cubic of the example,
            (x_n - x_1 z)(2wV + sigma z)^2 - sigma g V x_1^2 = 0,
        and h = 2V x_1 / (2wV + sigma z).  The paper leaves the branch open ("upon
        choosing a specific branch").  Reading: the root with W = 2wV + sigma z > 0
        and W^2 > g h, i.e. the largest real root for sigma = +1 and the smallest
        for sigma = -1; it is the only root continuous with the equilibrium state
        under the sub-characteristic condition.  Roots come from the eigenvalues of
        the companion matrix (numpy), then two Newton polishing steps.
        """
        n, s, g = lat.axis[k], lat.sign[k], self.g
        x1, xn = x[0], x[1 + n]
        W0 = 2.0 * lat.w * V
        # cubic in z:  -x1 z^3 + (xn - 2 s W0 x1) z^2 + (2 s W0 xn - W0^2 x1) z + (W0^2 xn - s g V x1^2)
        c3 = -x1
        c2 = xn - 2.0 * s * W0 * x1
        c1 = 2.0 * s * W0 * xn - W0 ** 2 * x1
        c0 = W0 ** 2 * xn - s * g * V * x1 ** 2
        shp = x1.shape
        c3f = np.where(c3 == 0, 1.0, c3).ravel()
        comp = np.zeros((c3f.size, 3, 3))
        comp[:, 0, 0] = -(c2.ravel() / c3f)
        comp[:, 0, 1] = -(c1.ravel() / c3f)
        comp[:, 0, 2] = -(c0.ravel() / c3f)
        comp[:, 1, 0] = 1.0
        comp[:, 2, 1] = 1.0
        roots = np.linalg.eigvals(comp)  # (n, 3)
        real = np.abs(roots.imag) <= 1e-9 * (np.abs(roots.real) + V)
        zr = roots.real
        Wr = W0 + s * zr
        hr = 2.0 * V * x1.ravel()[:, None] / np.where(Wr == 0, 1.0, Wr)
        ok = real & (Wr > 0) & (hr > 0) & (Wr ** 2 > g * hr)
        if s > 0:
            z = np.max(np.where(ok, zr, -np.inf), axis=1)
        else:
            z = np.min(np.where(ok, zr, np.inf), axis=1)
        valid = ok.any(axis=1) & (x1.ravel() > 0)
        z = np.where(valid, z, 0.0).reshape(shp)
        valid = valid.reshape(shp)
        for _ in range(2):
            W = W0 + s * z
            P = (xn - x1 * z) * W ** 2 - s * g * V * x1 ** 2
            dP = -x1 * W ** 2 + 2.0 * s * (xn - x1 * z) * W
            step = np.where(valid & (dP != 0), P / np.where(dP == 0, 1.0, dP), 0.0)
            z = z - step
        W = W0 + s * z
        h = 2.0 * V * x1 / np.where(valid, W, 1.0)
        valid &= (W > 0) & (h > 0) & (W ** 2 > g * h)
        vel = []
        for j in range(self.d):
            vel.append(z if j == n else x[1 + j] / np.where(valid, x1, 1.0))
        return h, np.array(vel), valid

    def bregman(self, lat, V, k, u, feqk, e):
        """B_k = [g W dh^2 + 2 sigma g h' dh du_n + h' W' |du|^2] / (4V).

        dh = h' - h, du = u' - u (population state minus cell state); W and W' are
        2wV + sigma u_n at the cell and at the population state.  Derived from the
        Legendre form of B_k with s_k^* = g h^2 W / (4V); pinned by brute force.
        The offsets come from the increment form of the inversion: with
        x_1 = f_1 + e_1, g_n = e_n - e_1 u_n and W' = W + sigma dn,
            sigma g V (sigma dn f_1 - e_1 W)(f_1 W' + x_1 W) + (g_n - x_1 dn) W^2 W'^2 = 0
        (the cubic of the example minus its value at the cell state), refined by
        Newton from the root of the plain cubic; then du_t = (e_t - u_t e_1) / x_1
        and dh = 2V (e_1 W - sigma f_1 dn) / (W W').
        """
        n, s, g = lat.axis[k], lat.sign[k], self.g
        h = u[0]
        vel = u[1:] / h
        x = feqk + e
        hp0, velp0, valid = self.population_state(lat, V, k, x)
        W = 2.0 * lat.w * V + s * vel[n]
        f1, e1 = feqk[0], e[0]
        x1 = f1 + e1
        gn = e[1 + n] - e1 * vel[n]
        dn = np.where(valid, velp0[n] - vel[n], 0.0)
        for _ in range(3):
            Wp = W + s * dn
            A = s * dn * f1 - e1 * W
            Bq = f1 * Wp + x1 * W
            C = gn - x1 * dn
            Dq = W ** 2 * Wp ** 2
            P = s * g * V * A * Bq + C * Dq
            dP = g * V * f1 * (Bq + A) - x1 * Dq + 2.0 * s * C * W ** 2 * Wp
            dn = dn - np.where(valid & (dP != 0), P / np.where(dP == 0, 1.0, dP), 0.0)
        Wp = W + s * dn
        dh = 2.0 * V * (e1 * W - s * f1 * dn) / (W * np.where(valid, Wp, 1.0))
        hp = h + dh
        du = []
        x1s = np.where(valid, x1, 1.0)
        for j in range(self.d):
            du.append(dn if j == n else (e[1 + j] - vel[j] * e1) / x1s)
        du = np.array(du)
        du2 = np.sum(du ** 2, axis=0)
        B = (g * W * dh ** 2 + 2.0 * s * g * hp * dh * du[n] + hp * Wp * du2) / (4.0 * V)
        dv = np.concatenate([(g * dh - 0.5 * np.sum(du * (2.0 * vel + du), axis=0))[None], du])
        return B, dv, valid

    def admissible(self, u):
        return u[0] > 0

    def subcharacteristic(self, lat, V, u):
        h = u[0]
        vel = u[1:] / h
        ok = h > 0
        for k in range(lat.q):
            W = 2.0 * lat.w * V + lat.sign[k] * vel[lat.axis[k]]
            ok &= (W > 0) & (W ** 2 > self.g * h)
        return ok


class Euler:
    """Compressible Euler u = (rho, rho u_1..u_d, E) with p = (gamma-1)(E - rho|u|^2/2) (Sec. 6.3).

    Entropy (reading, the paper gives none for Euler): S = -rho s / (gamma - 1),
    s = ln p - gamma ln rho; v = ((gamma - s)/(gamma-1) - beta |u|^2/2, beta u, -beta),
    beta = rho / p.  Population state for axis n, sign sigma, W = 2wV + sigma u_n:
        x_1 = rho W / (2V), x_n = x_1 u_n + sigma p / (2V), x_t = x_1 u_t,
        x_E = (E W + sigma u_n p) / (2V).
    """

    name = "euler"

    def __init__(self, gamma, d=2):
        self.gamma = float(gamma)
        self.d = d
        self.M = d + 2

    def primitives(self, u):
        rho = u[0]
        vel = u[1:1 + self.d] / rho
        E = u[1 + self.d]
        p = (self.gamma - 1.0) * (E - 0.5 * rho * np.sum(vel ** 2, axis=0))
        return rho, vel, p

    def flux(self, u, j):
        rho, vel, p = self.primitives(u)
        E = u[1 + self.d]
        out = np.empty_like(u)
        out[0] = u[1 + j]
        out[1:1 + self.d] = u[1 + j] * vel
        out[1 + j] += p
        out[1 + self.d] = vel[j] * (E + p)
        return out

    def macro_entropy(self, u):
        rho, vel, p = self.primitives(u)
        s = np.log(p) - self.gamma * np.log(rho)
        return -rho * s / (self.gamma - 1.0)

    def entropy_variable(self, u):
        rho, vel, p = self.primitives(u)
        gm = self.gamma
        s = np.log(p) - gm * np.log(rho)
        beta = rho / p
        v1 = (gm - s) / (gm - 1.0) - 0.5 * beta * np.sum(vel ** 2, axis=0)
        return np.concatenate([v1[None], beta * vel, -beta[None]])

    def population_state(self, lat, V, k, x):
        """Invert f_k^eq(U) = x.

        u_t = x_t / x_1; the normal velocity z solves the quadratic obtained by
        eliminating rho, p and E from the four relations above:
            -(gamma+1) x_1 z^2 + (2 gamma x_n - 2 sigma W0 x_1) z
              + 2 sigma W0 x_n + (gamma-1) x_t^2 / x_1 - 2 (gamma-1) x_E = 0,
        W0 = 2wV; then p = 2 sigma V (x_n - x_1 z), rho = 2V x_1 / (W0 + sigma z).
        Branch (reading): the larger root for sigma = +1, the smaller for sigma = -1,
        kept only if rho, p > 0 and rho W^2 > gamma p (sub-characteristic).
        """
        n, s, gm = lat.axis[k], lat.sign[k], self.gamma
        W0 = 2.0 * lat.w * V
        x1, xn, xE = x[0], x[1 + n], x[1 + self.d]
        pos = x1 > 0
        x1s = np.where(pos, x1, 1.0)
        xt2 = np.zeros_like(x1)
        for j in range(self.d):
            if j != n:
                xt2 = xt2 + x[1 + j] ** 2
        A = -(gm + 1.0) * x1
        B = 2.0 * gm * xn - 2.0 * s * W0 * x1
        C = 2.0 * s * W0 * xn + (gm - 1.0) * xt2 / x1s - 2.0 * (gm - 1.0) * xE
        disc = B * B - 4.0 * A * C
        valid = pos & (disc >= 0)
        sq = np.sqrt(np.where(valid, disc, 0.0))
        # the two roots, written without cancellation: q = -(B + sign(B) sq) / 2
        qq = -0.5 * (B + np.where(B >= 0, 1.0, -1.0) * sq)
        Ar = np.where(A == 0, 1.0, A)
        qqs = np.where(qq == 0, 1.0, qq)
        r1 = qq / Ar
        r2 = C / qqs
        z = np.maximum(r1, r2) if s > 0 else np.minimum(r1, r2)
        W = W0 + s * z
        p = 2.0 * s * V * (xn - x1 * z)
        rho = 2.0 * V * x1 / np.where(W == 0, 1.0, W)
        valid &= (W > 0) & (rho > 0) & (p > 0) & (rho * W ** 2 > gm * p)
        vel = []
        for j in range(self.d):
            vel.append(z if j == n else x[1 + j] / x1s)
        return rho, np.array(vel), p, valid

    def bregman(self, lat, V, k, u, feqk, e):
        """B_k = x_1 [phi(a/b)/(gamma-1) + phi(1/b)] + rho x_1 |du|^2 / (2p) + sigma rho dp du_n / (2Vp).

        a = p'/p, b = rho'/rho, phi(z) = z - 1 - ln z, primes for the population
        state.  Derived from s_k(x) = -x_1 s(U_k) / (gamma-1); pinned by brute force.
        Offsets in increment form (x = f^eq + e, x_1 = f_1 + e_1, g_n = e_n - e_1 u_n):
            du_t = (e_t - u_t e_1) / x_1,   dp = 2 sigma V (g_n - x_1 dn),
            drho = 2V (e_1 W - sigma f_1 dn) / (W W'),
        and dn is the root near 0 of  qa dn^2 + qb dn + qc = 0, the energy relation
        minus its value at the cell state:
            qa = -V x_1 (gamma+1)/(gamma-1),
            qb = 2V x_1 u_n + (sigma P0 + P1 W + sigma p)/(gamma-1) + sigma (p + P0 + u_n P1),
            qc = -2V e_E + V [e_1 (u_n^2 + u_t'^2) + f_1 du_t (2 u_t + du_t)]
                 + P0 W/(gamma-1) + sigma u_n P0,
        P0 = 2 sigma V g_n, P1 = -2 sigma V x_1.  The plain inversion (population_state)
        decides validity and the branch; the increment form gives the offsets.
        """
        n, s, gm = lat.axis[k], lat.sign[k], self.gamma
        rho, vel, p = self.primitives(u)
        x = feqk + e
        _, _, _, valid = self.population_state(lat, V, k, x)
        W0 = 2.0 * lat.w * V
        un = vel[n]
        W = W0 + s * un
        f1, e1 = feqk[0], e[0]
        x1 = f1 + e1
        x1s = np.where(valid, x1, 1.0)
        gn = e[1 + n] - e1 * un
        du = [None] * self.d
        ut2p = np.zeros_like(x1)
        corr = np.zeros_like(x1)
        for j in range(self.d):
            if j != n:
                du[j] = (e[1 + j] - vel[j] * e1) / x1s
                ut2p = ut2p + (vel[j] + du[j]) ** 2
                corr = corr + f1 * du[j] * (2.0 * vel[j] + du[j])
        P0 = 2.0 * V * s * gn
        P1 = -2.0 * V * s * x1
        qa = -V * x1 * (gm + 1.0) / (gm - 1.0)
        qb = 2.0 * V * x1 * un + (s * P0 + P1 * W + s * p) / (gm - 1.0) + s * (p + P0 + un * P1)
        qc = -2.0 * V * e[1 + self.d] + V * (e1 * (un ** 2 + ut2p) + corr) + P0 * W / (gm - 1.0) + s * un * P0
        disc = qb * qb - 4.0 * qa * qc
        valid = valid & (disc >= 0)
        den = qb + np.where(qb >= 0, 1.0, -1.0) * np.sqrt(np.where(valid, disc, 0.0))
        dn = np.where(valid, -2.0 * qc / np.where(den == 0, 1.0, den), 0.0)
        du[n] = dn
        du = np.array(du)
        dp = P0 + P1 * dn
        Wp = W + s * dn
        drho = 2.0 * V * (e1 * W - s * f1 * dn) / (W * np.where(valid, Wp, 1.0))
        al = dp / p
        be = drho / rho
        zeta1 = (al - be) / (1.0 + be)          # a/b - 1
        zeta2 = -be / (1.0 + be)                # 1/b - 1
        with np.errstate(invalid="ignore", divide="ignore"):
            phi1 = zeta1 - np.log1p(zeta1)
            phi2 = zeta2 - np.log1p(zeta2)
            B = (x1 * (phi1 / (gm - 1.0) + phi2) + rho * x1 * np.sum(du ** 2, axis=0) / (2.0 * p)
                 + s * rho * dp * dn / (2.0 * V * p))
            # entropy-variable difference v(U_k) - v(u)
            beta = rho / p
            dbeta = beta * (be - al) / (1.0 + al)
            ds = np.log1p(al) - gm * np.log1p(be)
        velp = vel + du
        dkin = dbeta * np.sum(velp ** 2, axis=0) + beta * np.sum(du * (2.0 * vel + du), axis=0)
        dv1 = -ds / (gm - 1.0) - 0.5 * dkin
        dv = np.concatenate([dv1[None], dbeta * velp + beta * du, -dbeta[None]])
        return np.where(valid, B, 0.0), dv, valid

    def admissible(self, u):
        rho, vel, p = self.primitives(u)
        return (rho > 0) & (p > 0)

    def subcharacteristic(self, lat, V, u):
        rho, vel, p = self.primitives(u)
        ok = (rho > 0) & (p > 0)
        c = np.sqrt(np.where(ok, self.gamma * p / np.where(rho > 0, rho, 1.0), 0.0))
        for k in range(lat.q):
            W = 2.0 * lat.w * V + lat.sign[k] * vel[lat.axis[k]]
            ok &= W > c
        return ok


def bregman_sum(lat, sys, V, u, feq, d, t):
    """F(t) = sum_k B_k(f_k^eq + t d_k) and F'(t) = sum_k (v(U_k) - v(u)) . d_k, per cell.

    ``t`` is an array over cells.  Also returns a validity mask (every
    population of the cell has a population state on the convex branch).
    """
    F = np.zeros(u.shape[1:])
    dF = np.zeros(u.shape[1:])
    ok = np.ones(u.shape[1:], bool)
    for k in range(lat.q):
        Bk, dvk, vk = sys.bregman(lat, V, k, u, feq[k], t * d[k])
        F = F + Bk
        dF = dF + np.sum(dvk * d[k], axis=0)
        ok &= vk
    return F, dF, ok


def kinetic_entropy_sum(lat, sys, V, f):
    """Sigma(f) = sum_k s_k(f_k) per cell, as S(u) + F(1) (Bregman identity, Sec. 4)."""
    u = f.sum(axis=0)
    feq = equilibrium(lat, sys, V, u)
    F, _, ok = bregman_sum(lat, sys, V, u, feq, f - feq, np.ones(u.shape[1:]))
    return sys.macro_entropy(u) + F, ok
