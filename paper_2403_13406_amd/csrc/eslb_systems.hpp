// Per-node physics of the fourth-order entropy-stable lattice Boltzmann scheme,
// device side (gfx950, binary64).
//
// Sec. 1.2: equilibria f_k^eq = w u + sigma_k phi^{n_k}(u) / (2V), w = 1/q, with
// n_k the axis and sigma_k the sign of V_k (D1Q2: +, -; D2Q4: +x, +y, -x, -y).
//
// Entropy-limited relaxation (Sec. 4, eq. variableOmegaProblem; Sec. 5.1): with
// d = f - f^eq and lambda = omega - 1, Sigma(f^eq + t d) = S(u) + F(t),
//   F(t) = sum_k B_k(t),  B_k = Bregman divergence of s_k between f_k^eq + t d_k
// and f_k^eq.  omega solves F(-lambda) = F(1).  B_k is evaluated from the
// "population state" offset U_k - u, where f_k^eq(U_k) = f_k^eq(u) + t d_k, and
// that offset is obtained from an equation written in increments (e = t d) so
// that nothing O(1) cancels: the distance from equilibrium is factored out.
//
// Each system provides
//   flux(u, j, phi)        phi^j(u)
//   prepare(u, c)          node constants; false if u is inadmissible
//   subchar(c)             convexity (sub-characteristic) condition at the node
//   macro_entropy(c)       S(u)
//   bregman<k>(c, feq_k, e, B, dv)   B_k and v(U_k) - v(u); false outside the domain
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <math.h>

namespace eslb {

struct Phys {
  double V;      // kinetic velocity
  double inv2V;  // 1 / (2V)
  double w;      // 1 / q
  double W0;     // 2 w V
  double p0, p1; // system parameters (a_x,a_y | b_x,b_y | g | gamma)
  double p2;     // derived: 1/(gamma-1) for Euler
  double omega;  // fixed relaxation parameter
  double V2;     // 2V
  double q0;     // derived: -V (gamma+1)/(gamma-1) for Euler
};

// Reciprocal from the hardware estimate (relative error below 2^-24 on gfx950,
// measured) refined by one third-order step: with e = 1 - x r,
// r <- r (1 + e + e^2) leaves e^3 < 2^-72, so the result is within rounding.
// Arguments here are O(1) positive or negative normal numbers.
__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Reciprocal refined by one Newton step (relative error about 2^-48), where that
// is all the precision the result needs.
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// sqrt of a positive normal number: hardware rsq estimate (relative error below
// 2^-24), one Goldschmidt refinement of (sqrt x, 1/(2 sqrt x)) (error ~2^-48)
// and a final residual correction s + (x - s^2)/(2 sqrt x) (error ~2^-96).
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  const double d = fma(-s, s, x);
  return fma(d, h, s);
}

// phi(z) = z - log1p(z) in three tiers, chosen per pair of arguments (the Euler
// evaluation's za, zb).  For |z| < 2^-7 (increments near equilibrium)
// phi(z) = z^2 g(z) with g(z) = sum_j (-1)^j z^j / (j + 2): its Taylor polynomial
// to z^4 for |z| <= 2^-10.5 (phi_taylor4), otherwise its Chebyshev-economised
// degree-6 polynomial on [-2^-7, 2^-7] (phi_poly; relative error below 2^-52 in
// binary64; no cancellation between z and log1p(z)); beyond, z - log1p_far(z).
__device__ __forceinline__ double phi_poly(double z) {
  double g = 0.12501220790442075;
  g = fma(g, z, -0.14286901156622775);
  g = fma(g, z, 0.16666666620096096);
  g = fma(g, z, -0.199999999637788);
  g = fma(g, z, 0.25000000000000566);
  g = fma(g, z, -0.3333333333333361);
  g = fma(g, z, 0.5);
  return (z * z) * g;
}

// log(1 + z) for z > -1 outside the series range: 1 + z = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),
// s = (m - 1)/(m + 1), |s| <= 0.1716, summed to s^21 (truncation below 1e-18);
// ln 2 split so that e ln2_hi is exact; the rounding of 1 + z corrected to first
// order by c/(1 + z), c = z - ((1 + z) - 1).  Few live values: it sits in the
// cold branch of every Bregman term, where the library log1p costs the
// relaxation kernels spilled registers.
__device__ inline double log1p_far(double z) {
  const double u = 1.0 + z;
  const double c = z - (u - 1.0);
  int e;
  double m = frexp(u, &e);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double s = (m - 1.0) * rcp(m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, s2, 1.0 / 19.0);
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  const double de = (double)e;
  const double rest = fma(de, 0x1.a39ef35793c76p-33, fma(2.0 * s, p, c * rcp(u)));
  return fma(de, 0x1.62e42fee00000p-1, rest);
}

// phi(z) = z^2 g(z) for |z| <= 2^-10.5 from the Taylor polynomial of g to z^4
// (truncation below 2 |z|^5 / 7 < 2^-54 relative)
__device__ __forceinline__ double phi_taylor4(double z) {
  double g = 1.0 / 6.0;
  g = fma(g, z, -0.2);
  g = fma(g, z, 0.25);
  g = fma(g, z, -1.0 / 3.0);
  g = fma(g, z, 0.5);
  return (z * z) * g;
}

// Bound of the Taylor tier of phi (and of the series reciprocal below).
constexpr double kPhiTaylor = 0x1.6a09e667f3bcdp-11;  // 2^-10.5

// phi for a pair outside the Taylor tier: the economised polynomial for |z| < 2^-7,
// otherwise z - log1p_far(z)
__device__ __forceinline__ void phi_pair_wide(double za, double zb, double& pa, double& pb) {
  if ((fabs(za) < 0.0078125) & (fabs(zb) < 0.0078125)) {
    pa = phi_poly(za);
    pb = phi_poly(zb);
  } else {
    pa = za - log1p_far(za);
    pb = zb - log1p_far(zb);
  }
}

// 1/(1 + z) for |z| <= 2^-10.5 from its geometric series to z^3 (truncation
// below |z|^4 < 2^-42 relative: it enters F' and the gradient of omega only,
// which need no more; see the Euler evaluation)
__device__ __forceinline__ double recip1p_small(double z) {
  // 1 - z + z^2 - z^3 = (1 + z^2)(1 - z)
  const double a = fma(z, z, 1.0);
  return fma(-z, a, a);
}

// Threshold of the predictor's skip measure (z / m^2, see Euler2 and
// ShallowWater::skip_limit).
constexpr double kSkipZ = 0x1p-8;

template <int D> struct Lat;
template <> struct Lat<1> {
  static constexpr int Q = 2;
  __host__ __device__ static constexpr int axis(int) { return 0; }
  __host__ __device__ static constexpr int sign(int k) { return k == 0 ? 1 : -1; }
};
template <> struct Lat<2> {
  static constexpr int Q = 4;
  __host__ __device__ static constexpr int axis(int k) { return k & 1; }
  __host__ __device__ static constexpr int sign(int k) { return k < 2 ? 1 : -1; }
};

// ---------------------------------------------------------------- advection
// phi^j = a_j u, S = u^2/2; s_k(x) = x^2 / (2 w_k), w_k = w + sigma a_n / (2V)
// (Example "Linear transport equation", Sec. 1.2.1 and 1.2.2).
template <int D> struct Advection {
  static constexpr int kStageBlocks = 2;  // resident 256-thread blocks per CU asked of the stage kernel
  static constexpr int kRecBlocks = kStageBlocks;  // the same for its recording form
  static constexpr int kBatchBlocks = 2;  // the same for the batch stage kernel
  static constexpr bool kTolFromU = false;  // see stop_tol
  static constexpr bool kSweepFinite = false;  // see fsum
  static constexpr bool kLdsD = false;
  static constexpr bool kDot = false;
  static constexpr int M = 1, Q = Lat<D>::Q;
  struct Node { double u; };
  using Fast = Advection;  // no deferred branch (see ShallowWater::Fast)
  __device__ static bool pending(const Node&) { return false; }
  __device__ static double skip_limit(const Node&, const Phys&) { return -1.0; }  // no skip measure
  __device__ static double a(int j, const Phys& P) { return j == 0 ? P.p0 : P.p1; }
  __device__ static void flux(const double* u, int j, double* phi, const Phys& P) { phi[0] = a(j, P) * u[0]; }
  __device__ static bool prepare(const double* u, Node& c, const Phys&) { c.u = u[0]; return true; }
  __device__ static bool subchar(const Node&, const Phys& P) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < Q; ++k) ok &= P.w + Lat<D>::sign(k) * a(Lat<D>::axis(k), P) * P.inv2V > 0.0;
    return ok;
  }
  __device__ static double macro_entropy(const Node& c, const Phys&) { return 0.5 * c.u * c.u; }
  // (d phi^j / du)^T z
  __device__ static void fluxT(const Node&, int j, const double* z, double* out, const Phys& P) { out[0] = a(j, P) * z[0]; }
  template <int k, bool DV>
  __device__ static bool bregman(const Node&, const double*, const double* d, double t, double& B, double* dv,
                                 const Phys& P, double /*zlim: no skip measure*/, bool& small) {
    small = false;
    const double wk = P.w + Lat<D>::sign(k) * a(Lat<D>::axis(k), P) * P.inv2V;
    const double dU = t * d[0] / wk;
    B = 0.5 * wk * dU * dU;
    if (DV) dv[0] = dU;
    return wk > 0.0;
  }
};

// ---------------------------------------------------------------- Burgers
// phi^j = b_j u^2 / 2, S = u^2/2, s_k^*(p) = w p^2/2 + beta_k p^3 / (12V),
// beta_k = sigma_k b_{n_k} (Example "Burgers' equation"; Sec. 3.3 in 2D).
// Increment equation of the population state: (beta/4V) dU^2 + c1 dU - e = 0,
// c1 = w + beta u / (2V); B = dU^2 (w/2 + beta (3u + 2 dU) / (12V)).
template <int D> struct Burgers {
  static constexpr int kStageBlocks = 2;  // resident 256-thread blocks per CU asked of the stage kernel
  static constexpr int kRecBlocks = kStageBlocks;  // the same for its recording form
  static constexpr int kBatchBlocks = 2;  // the same for the batch stage kernel
  static constexpr bool kTolFromU = false;  // see stop_tol
  static constexpr bool kSweepFinite = false;  // see fsum
  static constexpr bool kLdsD = false;
  static constexpr bool kDot = false;
  static constexpr int M = 1, Q = Lat<D>::Q;
  struct Node { double u; };
  using Fast = Burgers;  // no deferred branch (see ShallowWater::Fast)
  __device__ static bool pending(const Node&) { return false; }
  __device__ static double skip_limit(const Node&, const Phys&) { return -1.0; }  // no skip measure
  __device__ static double b(int j, const Phys& P) { return j == 0 ? P.p0 : P.p1; }
  __device__ static void flux(const double* u, int j, double* phi, const Phys& P) { phi[0] = 0.5 * b(j, P) * u[0] * u[0]; }
  __device__ static bool prepare(const double* u, Node& c, const Phys&) { c.u = u[0]; return true; }
  __device__ static bool subchar(const Node& c, const Phys& P) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < Q; ++k) ok &= P.w + Lat<D>::sign(k) * b(Lat<D>::axis(k), P) * c.u * P.inv2V > 0.0;
    return ok;
  }
  __device__ static double macro_entropy(const Node& c, const Phys&) { return 0.5 * c.u * c.u; }
  __device__ static void fluxT(const Node& c, int j, const double* z, double* out, const Phys& P) {
    out[0] = b(j, P) * c.u * z[0];
  }
  template <int k, bool DV>
  __device__ static bool bregman(const Node& c, const double*, const double* d, double t, double& B, double* dv,
                                 const Phys& P, double /*zlim: no skip measure*/, bool& small) {
    small = false;
    const double beta = Lat<D>::sign(k) * b(Lat<D>::axis(k), P);
    const double e = t * d[0];
    const double c1 = P.w + beta * c.u * P.inv2V;
    const double disc = c1 * c1 + 2.0 * beta * e * P.inv2V;
    const bool ok = (c1 > 0.0) && (disc > 0.0);
    const double dU = 2.0 * e * rcp(c1 + sqrt_pos(ok ? disc : c1 * c1));
    B = dU * dU * (0.5 * P.w + beta * (3.0 * c.u + 2.0 * dU) * (P.inv2V * (1.0 / 6.0)));
    if (DV) dv[0] = dU;
    return ok;
  }
};

// ---------------------------------------------------------------- shallow water
// u = (h, h u_1..u_D), S = h|u|^2/2 + g h^2/2, v = (g h - |u|^2/2, u)
// (Example "Shallow water system"; D2Q4 by the same construction).  For
// velocity k (axis n, sign sigma), W = 2wV + sigma u_n:
//   f^eq_1 = h W / (2V), f^eq_n = f^eq_1 u_n + sigma g h^2 / (4V), f^eq_t = f^eq_1 u_t,
//   s_k^* = g h^2 W / (4V).
// Increment equation for dn = u'_n - u_n (x = f^eq + e, x_1 = f^eq_1 + e_1,
// g_n = e_n - e_1 u_n, W' = W + sigma dn):
//   sigma g V (sigma dn f^eq_1 - e_1 W)(f^eq_1 W' + x_1 W) + (g_n - x_1 dn) W^2 W'^2 = 0,
// the cubic of the example with its O(1) part cancelled exactly; Newton from
// dn = 0 follows the branch with W'^2 > g h' (the physical one).  Then
//   du_t = (e_t - u_t e_1) / x_1,  dh = 2V (e_1 W - sigma f^eq_1 dn) / (W W'),
//   B = [g W dh^2 + 2 sigma g h' dh dn + h' W' |du|^2] / (4V).
// Admissibility of a root dn of the shallow-water population-state cubic:
// W' = W + sigma dn > 0, h' = h + dh > 0, W'^2 > g h', x_1 > 0.
__device__ inline bool sw_root_admissible(double dn, double W, double s, double e1, double f1, double x1, double h,
                                          double g, double V) {
  const double Wp = W + s * dn;
  const double hp = h + 2.0 * V * (e1 * W - s * f1 * dn) * rcp(W * Wp);
  return (x1 > 0.0) & (Wp > 0.0) & (hp > 0.0) & (Wp * Wp > g * hp);
}

// The branch rule on the population-state cubic P3 x^3 + P2 x^2 + P1 x + P0
// (P3 = -x_1 W^2 < 0), for the rare nodes where Newton from the cell state is not
// trustworthy: the extreme admissible real root -- largest for sigma = +1,
// smallest for sigma = -1 -- or NaN when there is none (the population state is
// then outside the domain).  With one real root (negative discriminant) it is
// bracketed by the Cauchy bound U = 1 + max |P_i / P3| (P(-U) > 0 > P(U)) and
// found by Newton safeguarded with bisection; with three, Newton from +-U runs
// monotonically onto the extreme one, and if that one is not admissible the
// other two come from the deflated quadratic.  No transcendental functions.
__device__ inline double sw_branch_root(double P0, double P1, double P2, double P3, double W, double s, double e1,
                                        double f1, double x1, double h, double g, double V) {
  const double i3 = rcp(P3);
  const double U = 1.0 + fmax(fabs(P2 * i3), fmax(fabs(P1 * i3), fabs(P0 * i3)));
  const double disc = 18.0 * P3 * P2 * P1 * P0 - 4.0 * P2 * P2 * P2 * P0 + P2 * P2 * P1 * P1 -
                      4.0 * P3 * P1 * P1 * P1 - 27.0 * P3 * P3 * P0 * P0;
  if (disc < 0.0) {
    double lo = -U, hi = U, x = 0.0;
    bool conv = false;
#pragma unroll 1
    for (int it = 0; it < 200; ++it) {
      const double Pv = P0 + x * (P1 + x * (P2 + x * P3));
      if (Pv > 0.0) {
        lo = x;
      } else {
        hi = x;
      }
      const double dP = P1 + x * (2.0 * P2 + 3.0 * P3 * x);
      double xn = x - Pv / dP;
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      const double st = xn - x;
      x = xn;
      if (!(fabs(st) > 0x1p-40 * fabs(x)) || !((hi - lo) > 0x1p-40 * fabs(x))) {
        conv = true;
        break;
      }
    }
    return (conv && sw_root_admissible(x, W, s, e1, f1, x1, h, g, V)) ? x : NAN;
  }
  double x = s * U;
#pragma unroll 1
  for (int it = 0; it < 200; ++it) {
    const double st = (P0 + x * (P1 + x * (P2 + x * P3))) / (P1 + x * (2.0 * P2 + 3.0 * P3 * x));
    x -= st;
    if (!(fabs(st) > 0x1p-40 * fabs(x))) break;
  }
  if (sw_root_admissible(x, W, s, e1, f1, x1, h, g, V)) return x;
  const double B1 = P2 + P3 * x, C1 = P1 + B1 * x;
  const double dq = B1 * B1 - 4.0 * P3 * C1;
  double best = NAN;
  if (dq >= 0.0) {
    const double qq = -0.5 * (B1 + copysign(sqrt(dq), B1));
    const double cand[2] = {qq * i3, C1 / qq};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double y = cand[i];
      if (isfinite(y) && sw_root_admissible(y, W, s, e1, f1, x1, h, g, V) &&
          (isnan(best) || (s > 0.0 ? y > best : y < best)))
        best = y;
    }
  }
  if (isfinite(best)) {
#pragma unroll
    for (int it = 0; it < 2; ++it)
      best -= (P0 + best * (P1 + best * (P2 + best * P3))) / (P1 + best * (2.0 * P2 + 3.0 * P3 * best));
  }
  return best;
}

template <int D> struct ShallowWaterFast;

template <int D> struct ShallowWater {
  // resident 256-thread blocks per CU asked of the stage kernel (waves per SIMD):
  // 2D at three (168 VGPRs; the spills cost less than the third wave gains:
  // 512-instance ensemble at a tenth of its steps, batch 7.57 -> 6.84 s and the
  // per-instance loop 11.7 -> 11.2 s against two waves; four lose, 8.25 s)
  static constexpr int kStageBlocks = (D == 1) ? 4 : 3;
  static constexpr int kRecBlocks = kStageBlocks;  // the same for its recording form
  static constexpr int kBatchBlocks = 3;  // the same for the batch stage kernel
  static constexpr bool kTolFromU = false;  // see stop_tol
  static constexpr bool kSweepFinite = false;  // see fsum
  static constexpr bool kLdsD = false;
  static constexpr bool kDot = false;
  static constexpr int M = D + 1, Q = Lat<D>::Q;
  // rule: set by the Fast variant's evaluations where Newton alone did not give
  // the branch root (the node is then relaxed again with the branch rule)
  struct Node { double h, vel[D]; mutable bool rule; };
  // Fast: the same evaluations without the branch rule (sw_branch_root).  The
  // rule is needed far from the cell state only; inlined into every evaluation it
  // costs the hot path registers and code, so relax_node runs the root search
  // with Fast and, on the rare nodes that flag it, once more with the rule
  // (measured on D2Q4: SW2D pass -1%, batched ensemble -2.6%; on D1Q2 it gained
  // nothing, so there the rule stays inline).
  using Fast = typename std::conditional<D == 2, ShallowWaterFast<D>, ShallowWater<D>>::type;
  __device__ static bool pending(const Node&) { return false; }  // this variant applies the rule itself
  // skip measure of the predictor (see Euler2): |dh|/h, |e_1|/f_1 and
  // |dn|/W at t = -1 against 2^-8 m^2, m = 1 - g h / W_min^2; on oracle roots the
  // prediction stays at the rounding floor up to z / m^2 ~ 2^-7 (D = 1 and 2)
  __device__ static double skip_limit(const Node& c, const Phys& P) {
    double vmax = fabs(c.vel[0]);
    if (D == 2) vmax = fmax(vmax, fabs(c.vel[D - 1]));
    const double Wmin = P.W0 - vmax;
    const double m = 1.0 - P.p0 * c.h * rcp(Wmin * Wmin);
    return (Wmin > 0.0 && m > 0.0) ? kSkipZ * m * m : -1.0;
  }
  __device__ static void flux(const double* u, int j, double* phi, const Phys& P) {
    const double h = u[0];
    const double uj = u[1 + j] * rcp(h);
    phi[0] = u[1 + j];
#pragma unroll
    for (int i = 0; i < D; ++i) phi[1 + i] = u[1 + i] * uj;
    phi[1 + j] += 0.5 * P.p0 * h * h;
  }
  __device__ static bool prepare(const double* u, Node& c, const Phys&) {
    c.h = u[0];
    c.rule = false;
    const double ih = rcp(u[0]);
#pragma unroll
    for (int i = 0; i < D; ++i) c.vel[i] = u[1 + i] * ih;
    return u[0] > 0.0;
  }
  __device__ static bool subchar(const Node& c, const Phys& P) {
    bool ok = c.h > 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const double W = P.W0 + Lat<D>::sign(k) * c.vel[Lat<D>::axis(k)];
      ok &= (W > 0.0) && (W * W > P.p0 * c.h);
    }
    return ok;
  }
  __device__ static double macro_entropy(const Node& c, const Phys& P) {
    double v2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) v2 += c.vel[i] * c.vel[i];
    return 0.5 * c.h * v2 + 0.5 * P.p0 * c.h * c.h;
  }
  // phi^j = (m_j, m_i m_j / h + delta_ij g h^2 / 2): transposed Jacobian times z
  __device__ static void fluxT(const Node& c, int j, const double* z, double* out, const Phys& P) {
    double zv = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) zv += z[1 + i] * c.vel[i];
    const double vj = c.vel[j];
    out[0] = -vj * zv + P.p0 * c.h * z[1 + j];
#pragma unroll
    for (int l = 0; l < D; ++l) out[1 + l] = vj * z[1 + l] + (l == j ? z[0] + zv : 0.0);
  }
  template <int k, bool DV, bool Rule = true>
  __device__ static bool bregman(const Node& c, const double* feq, const double* d, double t, double& B, double* dv,
                                 const Phys& P, double zlim, bool& small) {
    constexpr int n = Lat<D>::axis(k);
    constexpr double s = Lat<D>::sign(k);
    const double g = P.p0, V = P.V;
    const double un = c.vel[n];
    const double W = P.W0 + s * un;
    const double f1 = feq[0], e1 = t * d[0];
    const double x1 = f1 + e1;
    const double gn = t * (d[1 + n] - d[0] * un);
    const double W2 = W * W;
    // The cubic in monomial form P0 + P1 dn + P2 dn^2 + P3 dn^3 (with a = sigma f1,
    // A = a dn - e1 W, Bq = (f1 + x1) W + a dn, C = gn - x1 dn, Dq = W^2 W'^2);
    // P0 = O(e), P1 = f1 W^2 (g h - W^2) + O(e) < 0 in the sub-characteristic range.
    const double gV = s * g * V;
    const double a = s * f1, b = -e1 * W, cq = (f1 + x1) * W;
    const double P0 = gV * b * cq + gn * W2 * W2;
    const double P1 = gV * a * (b + cq) + W2 * W * (2.0 * s * gn - x1 * W);
    const double P2 = gV * a * a + W2 * (gn - 2.0 * s * x1 * W);
    const double P3 = -x1 * W2;
    // The root about dn = 0 by series reversion: with d0 = -P0/P1, q = P2 d0 / P1,
    // r = P3 d0^2 / P1, dn = d0 z and z = 1 - q z^2 - r z^3, i.e.
    //   z = 1 - q + 2q^2 - 5q^3 + 14q^4 - r + 5qr - 21q^2 r + 3r^2 + O(5)
    // (q of first order, r of second).  Near the cell state (|q| <= 2^-12,
    // |r| <= 2^-24) the fourth-order sum is the root to below 2^-52 relative and
    // no Newton step is taken.  Otherwise start from the third-order sum
    // d0 (1 - q + 2 q^2 - r) (error O(dn^4)) while its corrections are small changes
    // of the first Newton iterate from 0 (|q|, |r| <= 1/4), else from that iterate
    // itself, and run Newton, stopped once the error its recurrence leaves after a
    // step, |P''/(2P')| st^2, is below 2^-53 |dn|.
    const double rP1 = rcp(P1);
    const double d0 = -P0 * rP1;
    const double q = P2 * d0 * rP1, r = P3 * d0 * d0 * rP1;
    double dn;
    bool conv = false;
    if ((fabs(q) <= 0x1p-12) & (fabs(r) <= 0x1p-24)) {
      const double zq = fma(-q, fma(-q, fma(-q, fma(-14.0, q, 5.0), 2.0), 1.0), 1.0);
      const double zr = r * fma(-3.0, r, fma(-q, fma(-21.0, q, 5.0), 1.0));
      dn = d0 * (zq - zr);
      conv = true;
    } else {
      dn = (fabs(q) <= 0.25 && fabs(r) <= 0.25) ? d0 * (1.0 - q + (2.0 * q * q - r)) : d0;
#pragma unroll 1
      for (int it = 0; it < 12; ++it) {
        const double Pv = P0 + dn * (P1 + dn * (P2 + dn * P3));
        const double dP = P1 + dn * (2.0 * P2 + 3.0 * P3 * dn);
        const double rdP = rcp(dP);
        const double st = Pv * rdP;
        dn -= st;
        if (!(fabs(P2 + 3.0 * P3 * dn) * fabs(rdP) * st * st > 0x1p-53 * fabs(dn))) {
          conv = true;
          break;
        }
      }
    }
    // Far from the cell state (no convergence, |dn| > W/20, or a root outside the
    // admissible set) Newton may have run to another root of the cubic (near the
    // sonic point P1 -> 0): take the branch rule itself (sw_branch_root).
    double Wp = W + s * dn;
    double dh = 2.0 * V * (e1 * W - s * f1 * dn) * rcp(W * Wp);
    double hp = c.h + dh;
    if (!conv || fabs(dn) > 0.05 * W || !((x1 > 0.0) & (Wp > 0.0) & (hp > 0.0) & (Wp * Wp > g * hp))) {
      if constexpr (Rule) {
        dn = sw_branch_root(P0, P1, P2, P3, W, s, e1, f1, x1, c.h, g, V);
        Wp = W + s * dn;
        dh = 2.0 * V * (e1 * W - s * f1 * dn) * rcp(W * Wp);
        hp = c.h + dh;
      } else {
        c.rule = true;
        B = 0.0;
        small = false;
        if (DV)
#pragma unroll
          for (int m = 0; m < M; ++m) dv[m] = 0.0;
        return false;
      }
    }
    small = (fabs(dh) <= zlim * c.h) & (fabs(e1) <= zlim * f1) & (fabs(dn) <= zlim * W);
    double du2 = dn * dn;
    double kin = dn * (2.0 * un + dn);
    if (DV) dv[1 + n] = dn;
    if (D == 2) {
      constexpr int tt = 1 - n;
      const double ut = c.vel[tt];
      const double dt = t * (d[1 + tt] - ut * d[0]) * rcp(x1);
      du2 += dt * dt;
      kin += dt * (2.0 * ut + dt);
      if (DV) dv[1 + tt] = dt;
    }
    B = (g * W * dh * dh + 2.0 * s * g * hp * dh * dn + hp * Wp * du2) * (0.5 * P.inv2V);
    if (DV) dv[0] = g * dh - 0.5 * kin;
    return (x1 > 0.0) && (Wp > 0.0) && (hp > 0.0) && (Wp * Wp > g * hp) && isfinite(B);
  }
};

template <int D> struct ShallowWaterFast : ShallowWater<D> {
  using Base = ShallowWater<D>;
  __device__ static bool pending(const typename Base::Node& c) { return c.rule; }
  template <int k, bool DV>
  __device__ static bool bregman(const typename Base::Node& c, const double* feq, const double* d, double t, double& B,
                                 double* dv, const Phys& P, double zlim, bool& small) {
    return Base::template bregman<k, DV, false>(c, feq, d, t, B, dv, P, zlim, small);
  }
};

// ---------------------------------------------------------------- Euler (D2Q4)
// u = (rho, rho u, rho v, E), p = (gamma-1)(E - rho|u|^2/2) (Sec. 6.3).  Entropy
// S = -rho s/(gamma-1), s = ln p - gamma ln rho, v = ((gamma-s)/(gamma-1) -
// beta|u|^2/2, beta u, -beta), beta = rho/p; s_k^* is the mass component of
// f_k^eq.  For velocity k (axis n, sign sigma), W = 2wV + sigma u_n:
//   x_1 = rho W/(2V), x_n = x_1 u_n + sigma p/(2V), x_t = x_1 u_t,
//   x_E = (E W + sigma u_n p)/(2V).
// Increments: du_t = (e_t - u_t e_1)/x_1, dp = 2 sigma V (g_n - x_1 dn),
// drho = 2V (e_1 W - sigma f^eq_1 dn)/(W W'), and dn solves a A dn^2 + b dn + c = 0
// (energy relation, O(1) part removed); the root continuous from dn = 0 is the
// physical branch (rho' W'^2 > gamma p').  With al = dp/p, be = drho/rho and
// ds = log1p(al) - gamma log1p(be):
//   B = x_1 [((al - be)/(1+be) - ds)/(gamma-1) - be/(1+be)]
//       + rho x_1 |du|^2 / (2p) + sigma rho dp dn / (2V p).
// Where the population states at t = -1 stay close to the cell state, the
// cubic Hermite prediction of lambda is already within the root finder's
// stopping tolerance, and the confirming third evaluation of F is skipped.
// Measure: z = max over the q velocities, at t = -1, of |za|, |zb| (the
// relative pressure/density offsets of the thermal term) and |e_1| / f_1,
// against the sub-characteristic margin m = 1 - c^2 / W_min^2 (the Taylor
// radius of F in t shrinks with m); the prediction is taken when z <= 2^-8 m^2.
// On oracle roots over wide samples of states (density and pressure in
// [0.05, 20], velocities up to 99.9% of the sub-characteristic limit, relative
// offsets 1e-7 .. 1e-1) the prediction's effect on f' exceeded half the
// tolerance only from z / m^2 ~ 2^-7.5 on, and stays at the rounding floor
// below 2^-8; its error falls like (z / m^2)^6.

struct Euler2 {
  static constexpr int D = 2, M = 4, Q = 4;
  // resident 256-thread blocks per CU asked of the stage kernel: four waves per
  // SIMD (128 VGPRs), which the LDS-held d makes room for.  The hot path (the
  // predictor shortcut) does not spill; the safeguarded search does (its max|d|
  // and stop tolerance, a few dozen bytes per lane).  With the alternating row
  // order, whose passes leave the kernel waiting on memory more than on its
  // arithmetic, the fourth wave hides more of that wait: 4096^2 pass 816 -> 801 us
  // against three waves (168 VGPRs, no spills), same box.
  static constexpr int kStageBlocks = 4;
  // the recording form (the adjoint's reruns, which also store the pass input)
  // stays at three waves (168 VGPRs, no spills): at four, 1024^2 69.3 -> 71.3 us
  static constexpr int kRecBlocks = 3;
  static constexpr int kBatchBlocks = 2;  // batch stage kernel (d in registers: 2 waves)
  static constexpr bool kTolFromU = true;  // see stop_tol
  static constexpr bool kSweepFinite = true;  // eval leaves the finiteness of B to fsum
  static constexpr bool kLdsD = true;      // stage kernel keeps d in LDS (relax_node_lds)
  static constexpr bool kDot = true;       // fsum takes the F' term from bregman_dot
  // cell state: density, velocity, pressure, energy, 1/p, c^2 = gamma p / rho, and the
  // products the Bregman evaluations use: beta = rho/p, beta/2, beta/(2V), rho/(2V)
  struct Node { double rho, vel[2], p, E, ip, cs2, bet, hbet, sbet, rV; };
  using Fast = Euler2;  // no deferred branch (see ShallowWater::Fast)
  __device__ static bool pending(const Node&) { return false; }
  __device__ static void flux(const double* u, int j, double* phi, const Phys& P) {
    const double rho = u[0], ir = rcp(rho);
    const double vel[2] = {u[1] * ir, u[2] * ir};
    const double p = (P.p0 - 1.0) * (u[3] - 0.5 * rho * (vel[0] * vel[0] + vel[1] * vel[1]));
    flux_from(u, vel, p, j, phi);
  }
  // flux with the velocity and pressure of u given (as prepare and flux form them)
  __device__ static void flux_from(const double* u, const double* vel, double p, int j, double* phi) {
    const double uj = vel[j];
    phi[0] = u[1 + j];
    phi[1] = u[1] * uj;
    phi[2] = u[2] * uj;
    phi[1 + j] += p;
    phi[3] = uj * (u[3] + p);
  }
  __device__ static bool prepare(const double* u, Node& c, const Phys& P) {
    c.rho = u[0];
    const double ir = rcp(u[0]);
    c.vel[0] = u[1] * ir;
    c.vel[1] = u[2] * ir;
    c.E = u[3];
    c.p = (P.p0 - 1.0) * (u[3] - 0.5 * u[0] * (c.vel[0] * c.vel[0] + c.vel[1] * c.vel[1]));
    c.ip = rcp(c.p);
    c.cs2 = P.p0 * c.p * ir;
    c.bet = c.rho * c.ip;
    c.hbet = 0.5 * c.bet;
    c.sbet = P.inv2V * c.bet;
    c.rV = c.rho * P.inv2V;
    return (c.rho > 0.0) && (c.p > 0.0);
  }
  // limit of the skip measure: 2^-8 m^2, m = 1 - c^2/W_min^2 (negative: never skip)
  __device__ static double skip_limit(const Node& c, const Phys& P) {
    const double Wmin = P.W0 - fmax(fabs(c.vel[0]), fabs(c.vel[1]));
    const double m = 1.0 - c.cs2 * rcp1(Wmin * Wmin);  // a threshold: 2^-48 is plenty
    return (Wmin > 0.0 && m > 0.0) ? kSkipZ * m * m : -1.0;
  }
  __device__ static bool subchar(const Node& c, const Phys& P) {
    if (!((c.rho > 0.0) && (c.p > 0.0))) return false;
    const double cs2 = P.p0 * c.p / c.rho;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double W = P.W0 + Lat<2>::sign(k) * c.vel[Lat<2>::axis(k)];
      ok &= (W > 0.0) && (W * W > cs2);
    }
    return ok;
  }
  __device__ static double macro_entropy(const Node& c, const Phys& P) {
    return -c.rho * (log(c.p) - P.p0 * log(c.rho)) / (P.p0 - 1.0);
  }
  // phi^j = (m_j, m_i vel_j + delta_ij p, vel_j (E + p)): transposed Jacobian times z
  __device__ static void fluxT(const Node& c, int j, const double* z, double* out, const Phys& P) {
    const double gm1 = P.p0 - 1.0;
    const double vx = c.vel[0], vy = c.vel[1], vj = c.vel[j];
    const double H = (c.E + c.p) / c.rho;
    const double zv = z[1] * vx + z[2] * vy;
    const double A = z[1 + j] + z[3] * vj;
    const double dp_rho = 0.5 * gm1 * (vx * vx + vy * vy);
    out[0] = -vj * zv + dp_rho * A - z[3] * vj * H;
    out[1] = vj * z[1] - gm1 * vx * A + (j == 0 ? z[0] + zv + z[3] * H : 0.0);
    out[2] = vj * z[2] - gm1 * vy * A + (j == 1 ? z[0] + zv + z[3] * H : 0.0);
    out[3] = gm1 * z[1 + j] + P.p0 * vj * z[3];
  }

  // Population state of x = f^eq_k + t d_k, in increments from the cell state.
  // With e = t d the increment quadratic of the normal velocity dn simplifies
  // (the 2V x_1 u_n terms cancel):
  //   qa = -V x_1 (gamma+1)/(gamma-1),
  //   qb = sigma (gamma (t P0c + p) - 2V x_1 W)/(gamma-1),
  //   qc = t (qc1 + V dtn (2 u_t + du_t)),  du_t = t dtn / x_1,
  // with per-velocity constants gnd = d_n - u_n d_1, dtn = d_t - u_t d_1,
  // P0c = 2 sigma V gnd, qc1 = -2V d_E + V d_1 |u|^2 + P0c (W/(gamma-1) + sigma u_n).
  // Multiplied through by x_1 (qa/x_1 = q0 is a constant, qcx = x_1 qc has no
  // division), the quadratic needs one reciprocal, 1/(x_1 den), which also gives
  // 1/x_1.  The population state's density and pressure then follow without
  // division: x_1 = rho' W'/(2V) and f_1 = rho W/(2V) give
  //   zb = rho/rho' - 1 = (sigma rho dn/(2V) - e_1)/x_1,   al = p'/p - 1 = dp/p,
  //   za = (p'/p)(rho/rho') - 1 = al + zb + al zb.
  // The thermal part of B is x_1 [phi(za)/(gamma-1) + phi(zb)], phi(z) = z - log1p(z),
  // and ds = log1p(za) + (gamma-1) log1p(zb).  The entropy variables need
  // beta' = rho'/p' = beta/(1 + za): the one further reciprocal, only for F'.
  struct VelC { double W, gnd, dtn, P0c, qc1, qb0, qb1, cW, Vdtn, Q0, hd0, d0g; };
  template <int k>
  __device__ static VelC vel_consts(const Node& c, double un, double ut, double d0, double dn_, double dt_, double d3,
                                    const Phys& P) {
    constexpr double s = Lat<2>::sign(k);
    const double igm1 = P.p2, V = P.V, V2 = P.V2;
    VelC K;
    K.W = P.W0 + s * un;
    const double gnd = dn_ - un * d0;
    K.gnd = gnd;
    K.dtn = dt_ - ut * d0;
    K.P0c = s * V2 * gnd;
    K.qc1 = -V2 * d3 + V * d0 * (un * un + ut * ut) + K.P0c * (K.W * igm1 + s * un);
    const double sg = s * igm1 * P.p0;
    K.qb0 = sg * c.p;          // qb = qb0 + t qb1 - cW x_1
    K.qb1 = sg * K.P0c;
    K.cW = s * igm1 * V2 * K.W;
    K.Vdtn = V * K.dtn;
    // Q(u) = -|u|^2 d_1/2 + u_n d_n + u_t d_t - d_E (the F' term below)
    K.Q0 = fma(un, dn_, fma(ut, dt_, fma(-0.5 * d0, un * un + ut * ut, -d3)));
    K.hd0 = -0.5 * d0;
    K.d0g = d0 * igm1;
    return K;
  }
  // B_k(t) and (DV) F'-term (v(U_k) - v(u)) . d_k; false outside the convexity domain
  // B_k(t); DV: the F' term dvd = (v(U_k) - v(u)) . d_k; DVV: also the difference
  // v(U_k) - v(u) itself in dv (the adjoint's gradient of omega needs it)
  template <int k, bool DV, bool DVV = DV>
  __device__ static bool eval(const Node& c, double un, double ut, double f1, double d0, const VelC& K, double t,
                              double& B, double& dvd, double* dv, const Phys& P, double zlim, bool& small) {
    constexpr int n = Lat<2>::axis(k), tt = 1 - n;
    constexpr double s = Lat<2>::sign(k);
    const double igm1 = P.p2, V2 = P.V2;
    const double e1 = t * d0;
    const double x1 = f1 + e1;
    const double tdtn = t * K.dtn;
    const double qb = fma(-K.cW, x1, fma(t, K.qb1, K.qb0));
    const double qcx = t * fma(K.Vdtn, fma(2.0 * ut, x1, tdtn), K.qc1 * x1);
    // The root continuous from y = 0 of q0 y^2 + qb y + qcx = 0, y = x_1 dn.  Near
    // equilibrium eps = q0 qcx / qb^2 is small and y = -(qcx/qb) C(eps) with
    // C(eps) = 2/(1 + sqrt(1 - 4 eps)) = sum_j Cat_j eps^j (Catalan numbers), summed
    // to eps^4 for |eps| < 2^-11 (truncation below 43 |eps|^5 < 2^-49): one
    // reciprocal, 1/(x_1 qb), gives 1/qb and 1/x_1.  B needs no more: it is formed
    // from the increments with nothing O(1) cancelling, so a relative error e of dn
    // moves F by about 2e relative, and lambda by about e; near equilibrium
    // (|d| <= 2^-11 |f| here) that moves f^eq - lambda d by e |d|, below rounding.  Otherwise (also where x_1 qb
    // vanishes: eps is then not finite) the closed form with a square root.  (On
    // smooth 4096^2 Euler data |eps| stays below 2^-11.)
    const double aq = P.q0 * qcx;
    // once refined (relative error about 2^-48, the size of the series' truncation;
    // the closed form below has its own reciprocal)
    const double r = rcp1(x1 * qb);
    const double iqb = x1 * r;
    const double eps = aq * (iqb * iqb);
    double ix1, dn;  // 1/x_1, dn
    bool okd = true;
    if (fabs(eps) < 0x1p-11) {
      // 1 + eps (1 + eps (2 + eps (5 + 14 eps))), the innermost level as
      // eps (4 + 14 eps) + (eps + 2): inline constants only (no register to
      // materialise 5 in every evaluation)
      double cat = fma(eps, fma(eps, 14.0, 4.0), eps + 2.0);
      cat = fma(cat, eps, 1.0);
      cat = fma(cat, eps, 1.0);
      ix1 = qb * r;
      dn = -qcx * r * cat;
    } else {
      const double disc = fma(qb, qb, -4.0 * aq);
      okd = disc > 0.0;
      const double den = qb + copysign(okd ? sqrt_pos(disc) : 0.0, qb);
      const double r1 = rcp(x1 * den);
      ix1 = den * r1;
      dn = -2.0 * qcx * r1;
    }
    const double dt = tdtn * ix1;
    const double dp = fma(-s * V2 * x1, dn, t * K.P0c);
    const double Wp = K.W + s * dn;
    const double al = dp * c.ip;
    const double zb = fma(s * c.rV, dn, -e1) * ix1;
    const double za = fma(al, zb, al + zb);
    small = (fabs(za) <= zlim) & (fabs(zb) <= zlim) & (fabs(e1) <= zlim * f1);
    // phi(za), phi(zb), (DV) 1/(1 + za) = beta'/beta, and the domain conditions
    // rho' > 0 (zb > -1; with W' > 0, also x_1 > 0) and p' > 0 (al > -1).  In the
    // Taylor tier (|za|, |zb| <= 2^-10.5) rho'/rho and p'/p are within 2^-10 of 1,
    // so those conditions hold and are not tested.
    double pa, pb, ira = 0.0;
    bool okx;
    if ((fabs(za) <= kPhiTaylor) & (fabs(zb) <= kPhiTaylor)) {
      pa = phi_taylor4(za);
      pb = phi_taylor4(zb);
      if (DV) ira = recip1p_small(za);
      okx = okd;
    } else {
      phi_pair_wide(za, zb, pa, pb);
      // F' needs far less than full precision (its errors enter the predicted
      // lambda multiplied by lambda - 1): a once-refined reciprocal
      if (DV) ira = rcp1(1.0 + za);
      okx = okd & (x1 > 0.0) & (zb > -1.0) & (al > -1.0);
    }
    const double du2 = fma(dn, dn, dt * dt);
    const double pab = fma(pa, igm1, pb);  // phi(za)/(gamma-1) + phi(zb)
    B = fma(x1, fma(du2, c.hbet, pab), (s * c.sbet) * dp * dn);
    if (DV) {
      // entropy-variable difference v(U_k) - v(u): with ds = log1p(za) + (gamma-1) log1p(zb),
      //   v(U_k) - v(u) = (-ds/(gamma-1) - (beta'|u'|^2 - beta|u|^2)/2, beta' u' - beta u, -(beta' - beta)),
      // so its dot product with d_k is -ds d_1/(gamma-1) + beta' Q(u') - beta Q(u), Q as in vel_consts,
      // with Q(u') = Q(u) + dQ, dQ = dn (d_n - u_n d_1) + dt (d_t - u_t d_1) - |du|^2 d_1/2
      // and beta' Q(u') - beta Q(u) = beta (dQ - za Q(u)) / (1 + za)
      // ds = (za - pa) + (gamma-1) (zb - pb) = za + (gamma-1) (zb - pab)
      const double ds = fma(P.p0 - 1.0, zb - pab, za);
      const double dQ = fma(K.hd0, du2, fma(dn, K.gnd, dt * K.dtn));
      dvd = fma(-ds, K.d0g, (c.bet * ira) * fma(-za, K.Q0, dQ));
      if (DVV) {
        const double dbet = -c.bet * za * ira;
        const double unp = un + dn, utp = ut + dt;
        const double up2 = fma(unp, unp, utp * utp);
        const double dkin = fma(dbet, up2, c.bet * fma(dn, 2.0 * un + dn, dt * (2.0 * ut + dt)));
        dv[0] = fma(-ds, igm1, -0.5 * dkin);
        dv[1 + n] = fma(dbet, unp, c.bet * dn);
        dv[1 + tt] = fma(dbet, utp, c.bet * dt);
        dv[3] = -dbet;
      }
    }
    // W' > 0 and the sub-characteristic condition rho' W'^2 > gamma p', i.e.
    // W'^2 > c^2 (1 + za), as one test: W'|W'| > c^2 (1 + za) (1 + za > 0 where okx
    // holds).  A non-finite B is caught on the sum F by the sweeps (fsum, fsum_pm).
    return okx & (Wp * fabs(Wp) > fma(c.cs2, za, c.cs2));
  }
  template <int k, bool DV>
  __device__ static bool bregman(const Node& c, const double* feq, const double* d, double t, double& B, double* dv,
                                 const Phys& P, double zlim, bool& small) {
    constexpr int n = Lat<2>::axis(k), tt = 1 - n;
    // t-independent per-velocity constants; recomputed at every evaluation (the
    // opaque copy keeps the compiler from hoisting them: keeping them live for
    // all four velocities costs more registers than recomputing them)
    double d0 = d[0], dn_ = d[1 + n], dt_ = d[1 + tt], d3 = d[3];
    asm volatile("" : "+v"(d0), "+v"(dn_), "+v"(dt_), "+v"(d3));
    const double un = c.vel[n], ut = c.vel[tt];
    const VelC K = vel_consts<k>(c, un, ut, d0, dn_, dt_, d3, P);
    double dvd;
    return eval<k, DV, DV>(c, un, ut, feq[0], d0, K, t, B, dvd, dv, P, zlim, small);
  }
  // bregman returning the F' term (v(U_k) - v(u)) . d_k itself (fsum's form for this system)
  template <int k, bool DV>
  __device__ static bool bregman_dot(const Node& c, const double* feq, const double* d, double t, double& B,
                                     double& dvd, const Phys& P, double zlim, bool& small) {
    constexpr int n = Lat<2>::axis(k), tt = 1 - n;
    double d0 = d[0], dn_ = d[1 + n], dt_ = d[1 + tt], d3 = d[3];
    asm volatile("" : "+v"(d0), "+v"(dn_), "+v"(dt_), "+v"(d3));
    const double un = c.vel[n], ut = c.vel[tt];
    const VelC K = vel_consts<k>(c, un, ut, d0, dn_, dt_, d3, P);
    double dv[4];
    return eval<k, DV, false>(c, un, ut, feq[0], d0, K, t, B, dvd, dv, P, zlim, small);
  }
  // bregman for values just read from thread-private LDS slots (LdsSrc), the cell
  // velocity (vel) included: no copies, and nothing derived from them is kept
  // from one evaluation to the next
  template <int k, bool DV>
  __device__ static bool bregman_fresh(const Node& c, const double* vel, const double* feq, const double* d, double t,
                                       double& B, double& dvd, const Phys& P, double zlim, bool& small) {
    constexpr int n = Lat<2>::axis(k), tt = 1 - n;
    const VelC K = vel_consts<k>(c, vel[n], vel[tt], d[0], d[1 + n], d[1 + tt], d[3], P);
    double dv[4];
    return eval<k, DV, false>(c, vel[n], vel[tt], feq[0], d[0], K, t, B, dvd, dv, P, zlim,
                              small);
  }
  // The predictor's two samples for velocity k, t = +1 and t = -1 (the skip
  // measure at t = -1 only), from one read of its LDS slots: the per-velocity
  // constants are formed once and t is a constant in each evaluation.  The second
  // evaluation starts once the first is summed (interleaved, they need more
  // registers than the stage kernel's waves per SIMD allow).
  template <int k>
  __device__ static void pair_fresh(const Node& c, const double* vel, double f1, const double* d, const Phys& P,
                                    double zlim, double& F1, double& dF1, bool& ok1, double& Fm, double& dFm,
                                    bool& okm, bool& small) {
    constexpr int n = Lat<2>::axis(k), tt = 1 - n;
    double un = vel[n], ut = vel[tt], d0 = d[0], dn_ = d[1 + n], dt_ = d[1 + tt], d3 = d[3];
    const VelC K = vel_consts<k>(c, un, ut, d0, dn_, dt_, d3, P);
    double B, dvd, dv[4];
    bool sk;
    // the same sums as fsum's, so that the register path (relax_node) gives the same bits
    ok1 &= eval<k, true, false>(c, un, ut, f1, d0, K, 1.0, B, dvd, dv, P, -1.0, sk);
    F1 = (k == 0) ? B : F1 + B;  // the callers start the sums at 0
    dF1 = (k == 0) ? dvd : dF1 + dvd;
    asm volatile("" : "+v"(f1), "+v"(d0) : "v"(F1), "v"(dF1));
    okm &= eval<k, true, false>(c, un, ut, f1, d0, K, -1.0, B, dvd, dv, P, zlim, sk);
    small &= sk;
    Fm = (k == 0) ? B : Fm + B;
    dFm = (k == 0) ? dvd : dFm + dvd;
  }
};

// ------------------------------------------------------------- node relaxation

template <class S> struct Eq {
  static constexpr int Q = S::Q, M = S::M;
  // f_k^eq(u) = w u + sigma_k phi^{n_k}(u) / (2V)
  __device__ static void equilibrium(const double* u, double (&feq)[Q][M], const Phys& P) {
    double phx[M], phy[M];
    S::flux(u, 0, phx, P);
    if (Q == 4) S::flux(u, 1, phy, P);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int ax = (Q == 4) ? (k & 1) : 0;
#pragma unroll
      for (int m = 0; m < M; ++m) feq[k][m] = component(u[m], ax == 0 ? phx[m] : phy[m], k, P);
    }
  }
  // equilibrium from u with its velocity and pressure given (S::flux_from; the same
  // bits as equilibrium(u) when vel and p are the values prepare forms from u)
  __device__ static void equilibrium_from(const double* u, const double* vel, double p, double (&feq)[Q][M],
                                          const Phys& P) {
    double phx[M], phy[M];
    S::flux_from(u, vel, p, 0, phx);
    if (Q == 4) S::flux_from(u, vel, p, 1, phy);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int ax = (Q == 4) ? (k & 1) : 0;
#pragma unroll
      for (int m = 0; m < M; ++m) feq[k][m] = component(u[m], ax == 0 ? phx[m] : phy[m], k, P);
    }
  }
  // f^eq_{k,m} from u_m and phi^{n_k}_m (the same bits wherever it is formed)
  __device__ static double component(double um, double phim, int k, const Phys& P) {
    const double s = (k < Q / 2) ? P.inv2V : -P.inv2V;
    return P.w * um + s * phim;
  }
};

// max |d| over an array (a maximum of computed values)
template <class S>
__device__ __forceinline__ double max_abs(const double (&d)[S::Q][S::M]) {
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < S::Q; ++k)
#pragma unroll
    for (int j = 0; j < S::M; ++j) m = fmax(m, fabs(d[k][j]));
  return m;
}

// Where the root search reads d_k and the mass component of f^eq_k (the only
// component of f^eq the Bregman terms use): the arrays of node_split (RegSrc),
// or thread-private LDS slots (LdsSrc), so that only the velocity being
// evaluated holds them in registers.  get<k>(fence, ...) reads velocity k; for
// LDS the read address depends on `fence`, so the read cannot be moved ahead of
// whatever produced that value.
template <class S> struct RegSrc {
  static constexpr bool kFresh = false;  // values live in registers: S::bregman makes opaque copies
  const double (&feq)[S::Q][S::M];
  const double (&d)[S::Q][S::M];
  template <int k>
  __device__ __forceinline__ void get(double, double& f1, double (&dk)[S::M]) const {
    f1 = feq[k][0];
#pragma unroll
    for (int m = 0; m < S::M; ++m) dk[m] = d[k][m];
  }
  __device__ __forceinline__ double max_abs_feq() const { return max_abs<S>(feq); }
  __device__ __forceinline__ double dmax() const { return max_abs<S>(d); }
};

// LDS slots of one thread: slot j at p[j * kLdsStride] (blocks of kLdsStride
// threads, one slot of each thread side by side: conflict-free, and every slot
// an immediate offset from one address).  d_{k,m} at j = k M + m, the cell
// velocity at j = Q M + i (i < Q/2, the dimension).  18 slots for D2Q4^4: 18 KiB
// per 128-thread block, so eight blocks (four waves per SIMD) fit in a CU's LDS.
constexpr int kLdsStride = 128;
template <class S>
__host__ __device__ constexpr int lds_slots() { return S::Q * S::M + S::Q / 2; }

template <class S> struct LdsSrc {
  static constexpr bool kFresh = true;  // every get is a fresh read: S::bregman_fresh, no copies
  double* p;
  const double (&u)[S::M];  // the cell's conserved moments (registers)
  const Phys& P;
  template <int k>
  __device__ __forceinline__ void get(double fence, double& f1, double (&dk)[S::M], double (&vel)[S::Q / 2]) const {
    unsigned off = 0;
    asm volatile("" : "+v"(off) : "v"(fence));
    const double* q = p + off;
    // the mass of f^eq_k from u (phi^{n_k}_0 is the momentum u_{1+n_k}), as node_split forms it
    f1 = Eq<S>::component(u[0], u[1 + Lat<S::D>::axis(k)], k, P);
#pragma unroll
    for (int m = 0; m < S::M; ++m) dk[m] = q[(k * S::M + m) * kLdsStride];
#pragma unroll
    for (int i = 0; i < S::Q / 2; ++i) vel[i] = q[(S::Q * S::M + i) * kLdsStride];
  }
  __device__ __forceinline__ double max_abs_feq() const { return 0.0; }  // S::kTolFromU systems only
  __device__ __forceinline__ double dmax() const {
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < S::Q * S::M; ++j) m = fmax(m, fabs(p[j * kLdsStride]));
    return m;
  }
};

// F(t) = sum_k B_k and (DV) F'(t) = sum_k (v(U_k) - v(u)) . d_k, velocities k..Q-1.
// small: AND over the velocities of each system's "population state within
// zlim of the cell state" test (always false for systems without a skip measure
// and for zlim < 0).
template <class S, bool DV = true, int k = 0, class Src>
__device__ __forceinline__ bool fsum(const typename S::Node& c, const Src& src, double t, double& F, double& dF,
                                     const Phys& P, double zlim, bool& small, bool okacc = true) {
  if constexpr (k == S::Q) {
    if constexpr (S::kSweepFinite) return okacc & isfinite(F);
    return okacc;
  } else {
    double dv[S::M], B, f1, dk[S::M];
    bool sk;
    bool ok;
    if constexpr (Src::kFresh) {
      double vel[S::Q / 2], dvd;
      src.template get<k>(t, f1, dk, vel);
      ok = S::template bregman_fresh<k, DV>(c, vel, &f1, dk, t, B, dvd, P, zlim, sk);
      if (DV) dF = (k == 0) ? dvd : dF + dvd;  // the callers start the sums at 0
    } else if constexpr (S::kDot) {
      double dvd;
      src.template get<k>(t, f1, dk);
      ok = S::template bregman_dot<k, DV>(c, &f1, dk, t, B, dvd, P, zlim, sk);
      if (DV) dF = (k == 0) ? dvd : dF + dvd;
    } else {
      src.template get<k>(t, f1, dk);
      ok = S::template bregman<k, DV>(c, &f1, dk, t, B, dv, P, zlim, sk);
      if (DV) {
#pragma unroll
        for (int m = 0; m < S::M; ++m) dF += dv[m] * dk[m];
      }
    }
    small &= sk;
    okacc &= ok;
    if constexpr (S::kDot) {
      F = (k == 0) ? B : F + B;
    } else {
      F += B;
    }
    // Serialise the velocities: the next evaluation waits for this one's sums
    // and for its validity and skip tests, materialised here (left as booleans
    // combined at the end, their comparisons sink there and keep the operands of
    // every velocity live through the sweep).  Left free, the scheduler also
    // interleaves all q inversions for ILP and needs more registers than the
    // waves per SIMD allow (spills); in sequence they fit without spilling.
    double ts = t;
    int okv = okacc, smv = small;
    asm volatile("" : "+v"(ts), "+v"(okv), "+v"(smv) : "v"(F), "v"(dF));
    small = smv != 0;
    return fsum<S, DV, k + 1>(c, src, ts, F, dF, P, zlim, small, okv != 0);
  }
}

// Both predictor samples, velocity by velocity, for systems with S::pair_fresh
// reading an LdsSrc: F, F' at t = +1 (F1, dF1, ok1) and t = -1 (Fm, dFm, okm,
// small), each velocity's reads and evaluations after the previous one's sums
// and tests (materialised, as in fsum).
template <class S, int k = 0>
__device__ __forceinline__ void fsum_pm(const typename S::Node& c, const LdsSrc<S>& src, const Phys& P, double zlim,
                                        double& F1, double& dF1, bool& ok1, double& Fm, double& dFm, bool& okm,
                                        bool& small, double fence = 0.0) {
  if constexpr (k < S::Q) {
    double f1, dk[S::M], vel[S::Q / 2];
    src.template get<k>(fence, f1, dk, vel);
    S::template pair_fresh<k>(c, vel, f1, dk, P, zlim, F1, dF1, ok1, Fm, dFm, okm, small);
    double fn = 0.0;
    int o1 = ok1, om = okm, sm = small;
    asm volatile("" : "+v"(fn), "+v"(o1), "+v"(om), "+v"(sm) : "v"(F1), "v"(dF1), "v"(Fm), "v"(dFm));
    ok1 = o1 != 0;
    okm = om != 0;
    small = sm != 0;
    fsum_pm<S, k + 1>(c, src, P, zlim, F1, dF1, ok1, Fm, dFm, okm, small, fn);
  }
}

// Register-array form (the diagnostics and the adjoint's evaluations).
template <class S, bool DV = true>
__device__ __forceinline__ bool fsum(const typename S::Node& c, const double (&feq)[S::Q][S::M],
                                     const double (&d)[S::Q][S::M], double t, double& F, double& dF, const Phys& P,
                                     double zlim, bool& small) {
  return fsum<S, DV, 0>(c, RegSrc<S>{feq, d}, t, F, dF, P, zlim, small);
}

// u = sum_k f_k, f^eq(u), d = f - f^eq and nz = (some |d_{k,m}| > 0, i.e. max |d| > 0
// with NaN entries ignored as fmax ignores them).  max |d| itself is formed only
// where the root search needs it (Src::dmax).
template <class S>
__device__ __forceinline__ void node_split(const double (&f)[S::Q][S::M], double (&u)[S::M],
                                           double (&feq)[S::Q][S::M], double (&d)[S::Q][S::M], bool& nz,
                                           const Phys& P) {
  constexpr int Q = S::Q, M = S::M;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double acc = f[0][m];
#pragma unroll
    for (int k = 1; k < Q; ++k) acc += f[k][m];
    u[m] = acc;
  }
  Eq<S>::equilibrium(u, feq, P);
  nz = false;
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      d[k][m] = f[k][m] - feq[k][m];
      nz |= fabs(d[k][m]) > 0.0;
    }
}


// Tolerance of the stop rule: 2 eps (max |f^eq| + dmax), max |f^eq| + dmax being an
// upper bound of max(|f^eq|, |f|) within a factor 2.  Only the paths past the
// predictor shortcut need it, so it is formed there: from the f^eq of node_split
// (held by the source), or (S::kTolFromU) from f^eq rebuilt from the cell's u,
// so that only the mass components of f^eq stay live through the root search.
// The rebuild works on an opaque copy of u, so that the compiler cannot reuse
// (and keep live) node_split's f^eq instead; it gives the same bits.
template <class S, class Src>
__device__ __forceinline__ double stop_tol(const Src& src, double dmax, const double (&u)[S::M], const Phys& P) {
  double femax;
  if constexpr (S::kTolFromU) {
    double uu[S::M], feq[S::Q][S::M];
#pragma unroll
    for (int m = 0; m < S::M; ++m) {
      uu[m] = u[m];
      asm volatile("" : "+v"(uu[m]));
    }
    Eq<S>::equilibrium(uu, feq, P);
    femax = max_abs<S>(feq);
  } else {
    femax = src.max_abs_feq();
  }
  return 2.0 * 2.220446049250313e-16 * (femax + dmax);
}

// lambda = omega - 1 solving F(-lambda) = F(1) (eq. variableOmegaProblem in the
// Bregman form).  F is sampled with its derivative at t = 1 and t = -1 (lambda = 1);
// the cubic Hermite model of G(t) = F(t)/t^2 on [-1, 1] built from those four
// numbers is fourth-order accurate in the distance from equilibrium and predicts
// lambda; one more sample of F there gives a Newton correction (with the model's
// derivative, which is accurate to third order), and if that correction no longer
// moves f^eq - lambda d beyond rounding (2 eps max|f|) it is the root.  Otherwise
// (far from equilibrium, domain edges) a safeguarded Newton iteration with a
// bisection bracket takes over.  fallback = true when no root lies inside the
// convexity domain (omega = 1 then).
template <class S, class Src>
__device__ inline double entropic_lambda(const typename S::Node& c, const Src& src, const double (&u)[S::M],
                                         const Phys& P, bool& fallback) {
  fallback = false;
  double F1 = 0.0, dF1 = 0.0;
  bool small = true;  // all population states at t = -1 within the skip measure
  bool unused = true;
  double Fm = 0.0, dFm = 0.0;
  bool okm = true;
  if constexpr (Src::kFresh) {
    // both samples in one sweep; the t = -1 one is discarded where t = +1 is outside the domain
    bool ok1 = true;
    fsum_pm<S>(c, src, P, S::skip_limit(c, P), F1, dF1, ok1, Fm, dFm, okm, small);
    if constexpr (S::kSweepFinite) {
      ok1 &= isfinite(F1);
      okm &= isfinite(Fm);
    }
    if (!ok1) {
      // d = 0 exactly: omega = 2 with no search (the callers that test d before
      // the search never get here with it)
      if (!(src.dmax() > 0.0)) return 1.0;
      fallback = !S::pending(c);
      return 0.0;
    }
    if (!(F1 > 0.0)) return 1.0;
  } else {
    // S::pending: an evaluation needs the branch rule this variant leaves out
    // (the caller relaxes the node again with it)
    if (!fsum<S>(c, src, 1.0, F1, dF1, P, -1.0, unused)) {
      fallback = !S::pending(c);
      return 0.0;
    }
    if (!(F1 > 0.0)) return 1.0;
    okm = fsum<S>(c, src, -1.0, Fm, dFm, P, S::skip_limit(c, P), small);
  }
  double lo = 0.0, hi = INFINITY, x = 1.0;
  bool hi_bad = false;
  {
    if (S::pending(c)) return 0.0;
    const double H = Fm - F1;
    if (okm && H == 0.0) return 1.0;
    if (!okm || H > 0.0) {
      hi = 1.0;
      hi_bad = !okm;
    } else {
      lo = 1.0;
    }
    double xn = okm ? 1.0 + H * rcp1(dFm) : NAN;  // Newton from lambda = 1 (H' = -F'(-1)); a start only
    if (okm) {
      const double G1 = F1, Gm = Fm, G1p = dF1 - 2.0 * F1, Gmp = dFm + 2.0 * Fm;
      const double cc = 0.25 * (G1p - Gmp);
      const double dd = 0.25 * ((G1p + Gmp) - (G1 - Gm));
      const double bb = 0.5 * (G1 - Gm) - dd;
      const double aa = 0.5 * (G1 + Gm) - cc;
      // Newton on lambda^2 g(lambda) = G1 from lambda = 1.  The model's root is
      // within |lambda - 1| of 1, and its second derivative over twice its first is
      // about 1/2, so the error after j steps is about 2 (|lambda - 1| / 2)^(2^j):
      // three steps leave it below 2^-55 wherever |lambda - 1| < 2^-6 (the
      // predictor's skip region and far beyond); the second and third are taken
      // only where the previous step was not already below 2^-26, or, where the
      // prediction is taken as the root (small), below 2^-22: the error after it is
      // then below 2^-45, and the update moves f^eq - lambda d by that times
      // |d| <= 2^-8 |f| about (the skip region): below rounding.  The reciprocals
      // need no more than 2^-48.
      // The first step is xn: at lambda = 1 the model takes G(-1) = Fm and its
      // derivative -G'(-1), so the step is 1 + (Fm - F1)/F'(-1).  Each further step
      // is taken only while the previous one was above the limit (after a step st
      // the error is about st^2 / 2).
      double lp = xn, pd = 1.0, rpd = 1.0, st = 0.0;
      const double st_lim = small ? 0x1p-22 : 0x1p-26;
      const auto newton = [&]() {
        const double g = aa + lp * (-bb + lp * (cc - dd * lp));
        const double gp = -bb + lp * (2.0 * cc - 3.0 * dd * lp);
        const double pv = lp * lp * g - G1;
        pd = 2.0 * lp * g + lp * lp * gp;
        rpd = rcp1(pd);
        st = pv * rpd;
        lp -= st;
      };
      newton();
      if (!(fabs(st) <= st_lim)) {
        newton();
        if (!(fabs(st) <= st_lim)) newton();
      }
      if (isfinite(lp) && lp > lo && lp < hi && pd > 0.0) {
        // close to equilibrium the prediction is within the stopping tolerance
        if (small) return lp;
        double F3 = 0.0, dF3 = 0.0;
        const double dmax = src.dmax();
        const double tol = stop_tol<S>(src, dmax, u, P);
        const bool ok3 = fsum<S, false>(c, src, -lp, F3, dF3, P, -1.0, unused);
        if (S::pending(c)) return 0.0;
        const double H3 = F3 - F1;
        const double xc = lp - H3 * rpd;
        if (ok3 && isfinite(xc) && fabs(xc - lp) * dmax <= tol) return xc;
        if (!ok3 || H3 > 0.0) {
          if (lp <= hi) { hi = lp; hi_bad = !ok3; }
        } else {
          lo = fmax(lo, lp);
        }
        xn = (ok3 && isfinite(xc)) ? xc : lp;
      }
    }
    x = (isfinite(xn) && xn > lo && xn < hi) ? xn : (isinf(hi) ? 2.0 : 0.5 * (lo + hi));
  }
  const double dmax = src.dmax();
  const double tol = stop_tol<S>(src, dmax, u, P);
#pragma unroll 1
  for (int it = 0; it < 100; ++it) {
    double F = 0.0, dF = 0.0;
    bool unused = false;
    const bool ok = fsum<S>(c, src, -x, F, dF, P, -1.0, unused);
    if (S::pending(c)) return 0.0;
    const double H = F - F1, dH = -dF;
    if (ok && H == 0.0) return x;
    const bool above = !ok || (H > 0.0);
    if (above) {
      if (x <= hi) { hi = x; hi_bad = !ok; }
    } else {
      lo = fmax(lo, x);
    }
    const double xn = x - H / dH;
    // the bracket ends count as inside: at the root to rounding, x itself became
    // an end (H rounds to one side) and the Newton step rounds to x; a strict test
    // rejected that converged step and bisected the whole bracket again (up to ~45
    // evaluations on nodes near shocks, where the predictor is not taken)
    const bool newton_ok = ok && isfinite(xn) && (xn >= lo) && (xn <= hi);
    const double xnew = newton_ok ? xn : (isinf(hi) ? 2.0 * x : 0.5 * (lo + hi));
    if (newton_ok && fabs(xnew - x) * dmax <= tol) return xnew;
    if (!isinf(hi) && (hi - lo) * dmax <= tol) {
      if (hi_bad) {
        fallback = true;
        return 0.0;
      }
      return hi;
    }
    x = xnew;
  }
  return x;
}

enum : unsigned { FLAG_INADMISSIBLE = 1u, FLAG_NAN = 2u, FLAG_FALLBACK = 4u, FLAG_SUBCHAR = 8u };

// Relax one node in place.  mode 0: omega = P.omega (eq. relaxationDiscretizationOmega);
// mode 1: entropy-limited omega (eq. variableOmegaProblem).  Returns omega used;
// lam_out = the lambda = omega - 1 of the update, NaN where the root search fell
// back to omega = 1 (the adjoint then drops the grad-omega term).
template <class S>
__device__ __forceinline__ double relax_node(double (&f)[S::Q][S::M], int mode, const Phys& P, unsigned& flags,
                                    double& lam_out) {
  constexpr int Q = S::Q, M = S::M;
  double u[M], feq[Q][M], d[Q][M];
  bool nz;
  node_split<S>(f, u, feq, d, nz, P);
  // Both modes end with the same update f' = f^eq - lambda d, lambda = omega - 1
  // (for fixed omega, (1 - omega) f + omega f^eq written in d = f - f^eq): no
  // branch of the fixed mode keeps f or f^eq live through the entropic root search.
  bool fallback = false;
  double lam = P.omega - 1.0;
  if (mode != 0) {
    typename S::Node c;
    const bool adm = S::prepare(u, c, P);
    if (!adm) flags |= FLAG_INADMISSIBLE;
    // At equilibrium (d = 0, so f = f^eq exactly) omega = 2, the limit of the
    // root; the common update below then returns f^eq = f.
    lam = 1.0;
    if (nz) {
      fallback = !adm;
      lam = 0.0;
      const RegSrc<S> src{feq, d};
      if (adm) lam = entropic_lambda<typename S::Fast>(c, RegSrc<typename S::Fast>{feq, d}, u, P, fallback);
      if (S::Fast::pending(c)) lam = entropic_lambda<S>(c, src, u, P, fallback);
      if (fallback) {
        lam = 0.0;
        flags |= FLAG_FALLBACK;
      }
    }
  }
  // The root iteration only reads the mass component of each f^eq_k; rebuilding
  // f^eq from u here (rather than keeping all q*M values live through the
  // iteration) saves registers.  The empty asm makes u opaque so the compiler
  // recomputes instead of keeping the first copy alive; the rebuilt values are
  // the same bits.
#pragma unroll
  for (int m = 0; m < M; ++m) asm volatile("" : "+v"(u[m]));
  Eq<S>::equilibrium(u, feq, P);
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) f[k][m] = feq[k][m] - lam * d[k][m];
  lam_out = fallback ? NAN : lam;
  return lam + 1.0;
}

// relax_node with a fixed omega known at the call (no root search): the same
// arithmetic and bits as relax_node's fixed mode, without rebuilding f^eq.
template <class S>
__device__ __forceinline__ void relax_node_fixed(double (&f)[S::Q][S::M], const Phys& P) {
  constexpr int Q = S::Q, M = S::M;
  double u[M], feq[Q][M], d[Q][M];
  bool nz;
  node_split<S>(f, u, feq, d, nz, P);
  const double lam = P.omega - 1.0;
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) f[k][m] = feq[k][m] - lam * d[k][m];
}

template <class S>
__device__ __forceinline__ double relax_node(double (&f)[S::Q][S::M], int mode, const Phys& P, unsigned& flags) {
  double unused;
  return relax_node<S>(f, mode, P, flags, unused);
}

// relax_node for the stage kernel of systems with S::kLdsD: d and the cell
// velocity go to this thread's LDS slots (LdsSrc) right after node_split, and the
// root search reads them back one velocity at a time (the masses of f^eq it forms
// again from u), so that they do not occupy registers through it.  Same
// arithmetic and bits as relax_node.
template <class S>
__device__ __forceinline__ double relax_node_lds(double (&f)[S::Q][S::M], int mode, const Phys& P, unsigned& flags,
                                                 double& lam_out, double* slot) {
  constexpr int Q = S::Q, M = S::M;
  static_assert(S::kTolFromU, "LDS-held d needs the stop tolerance from u");
  double u[M];
  {
    double feq[Q][M], d[Q][M];
    bool nz;  // not needed here: see below
    node_split<S>(f, u, feq, d, nz, P);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
#pragma unroll
      for (int m = 0; m < M; ++m) slot[(k * M + m) * kLdsStride] = d[k][m];
    }
  }
  bool fallback = false;
  double lam = P.omega - 1.0;
  typename S::Node c;
  const bool adm = S::prepare(u, c, P);
  if (mode != 0) {
    if (!adm) flags |= FLAG_INADMISSIBLE;
#pragma unroll
    for (int i = 0; i < Q / 2; ++i) slot[(Q * M + i) * kLdsStride] = c.vel[i];
    // As relax_node: omega = 2 at equilibrium (d = 0), omega = 1 where the cell is
    // inadmissible and d is not 0, else the root.  The d = 0 test is left to the
    // paths where it decides something (inadmissible cells, and the root search's
    // out-of-domain exit: entropic_lambda), so admissible cells skip it: with d = 0
    // the search returns lambda = 1 at its F(1) > 0 test.
    const LdsSrc<S> src{slot, u, P};
    lam = 1.0;
    if (adm) {
      lam = entropic_lambda<S>(c, src, u, P, fallback);
    } else {
      fallback = src.dmax() > 0.0;
    }
    if (fallback) {
      lam = 0.0;
      flags |= FLAG_FALLBACK;
    }
  }
  // f^eq rebuilt from u with the velocity and pressure of prepare (the same bits
  // as node_split's; made opaque, as in relax_node, so that the compiler forms it
  // again instead of keeping node_split's live), d read back after lambda
  double vel[Q / 2], pc = c.p;
#pragma unroll
  for (int i = 0; i < Q / 2; ++i) {
    vel[i] = c.vel[i];
    asm volatile("" : "+v"(vel[i]));
  }
  asm volatile("" : "+v"(pc));
#pragma unroll
  for (int m = 0; m < M; ++m) asm volatile("" : "+v"(u[m]));
  double feq[Q][M];
  Eq<S>::equilibrium_from(u, vel, pc, feq, P);
  unsigned off = 0;
  asm volatile("" : "+v"(off) : "v"(lam));
  const double* q = slot + off;
#pragma unroll
  for (int k = 0; k < Q; ++k)
#pragma unroll
    for (int m = 0; m < M; ++m) f[k][m] = feq[k][m] - lam * q[(k * M + m) * kLdsStride];
  lam_out = fallback ? NAN : lam;
  return lam + 1.0;
}

// sum_k J_k^T y_k, J_k = d f_k^eq / du = w I + sigma_k (d phi^{n_k}/du) / (2V).
template <class S>
__device__ __forceinline__ void eq_jacobian_T(const typename S::Node& c, const double (&y)[S::Q][S::M],
                                              double (&out)[S::M], const Phys& P) {
  constexpr int Q = S::Q, M = S::M;
  double zx[M], zy[M], tx[M], ty[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double a = y[0][m];
#pragma unroll
    for (int k = 1; k < Q; ++k) a += y[k][m];
    out[m] = P.w * a;
    if (Q == 2) {
      zx[m] = y[0][m] - y[1][m];
    } else {
      zx[m] = y[0][m] - y[2][m];
      zy[m] = y[1][m] - y[3][m];
    }
  }
  S::fluxT(c, 0, zx, tx, P);
  if (Q == 4) S::fluxT(c, 1, zy, ty, P);
#pragma unroll
  for (int m = 0; m < M; ++m) out[m] += P.inv2V * (tx[m] + (Q == 4 ? ty[m] : 0.0));
}

template <class S, int k = 0>
__device__ __forceinline__ void dv_all(const typename S::Node& c, const double (&feq)[S::Q][S::M],
                                       const double (&d)[S::Q][S::M], double t, double (&dv)[S::Q][S::M],
                                       const Phys& P) {
  if constexpr (k < S::Q) {
    double B;
    bool unused;
    (void)S::template bregman<k, true>(c, feq[k], d[k], t, B, dv[k], P, -1.0, unused);
    // serialise the velocities, as in fsum (interleaved, they spill)
    double ts = t;
#pragma unroll
    for (int m = 0; m < S::M; ++m) asm volatile("" : "+v"(ts) : "v"(dv[k][m]));
    dv_all<S, k + 1>(c, feq, d, ts, dv, P);
  }
}

// gb[k] -= r dv_k(t) for every velocity, dv_k computed one velocity at a time.
template <class S, int k = 0>
__device__ __forceinline__ void sub_dv(const typename S::Node& c, const double (&feq)[S::Q][S::M],
                                       const double (&d)[S::Q][S::M], double t, double r, double (&gb)[S::Q][S::M],
                                       const Phys& P) {
  if constexpr (k < S::Q) {
    double B, dv[S::M];
    bool unused;
    (void)S::template bregman<k, true>(c, feq[k], d[k], t, B, dv, P, -1.0, unused);
    double ts = t;
#pragma unroll
    for (int m = 0; m < S::M; ++m) {
      gb[k][m] -= r * dv[m];
      asm volatile("" : "+v"(ts) : "v"(gb[k][m]));
    }
    sub_dv<S, k + 1>(c, feq, d, ts, r, gb, P);
  }
}

// Adjoint of one relaxation at a node: gbar (cotangent of the output) becomes
// hbar (cotangent of the input h), in place.
//   hbar_j = (1-omega) gbar_j + omega sum_k J_k^T gbar_k + grad_{h_j} omega * c,
//   c = sum_k (f^eq_k - h_k) . gbar_k,
//   grad_{h_j} omega = [(1-omega) dv_j(-lambda) + omega sum_k J_k^T dv_k(-lambda) - dv_j(1)] / F'(-lambda),
// dv_k(t) = v(U_k(t)) - v(u) (implicit function theorem on Sigma(R_omega h) = Sigma(h)).
// Two phases, so that the cotangent is not held through the root iteration:
// adjoint_root takes h to (u, d, lambda, omega, grad) -- the forward pass's
// relaxation, grad = omega depends on h -- and adjoint_apply updates gbar.
template <class S>
__device__ inline void adjoint_root(const double (&h)[S::Q][S::M], int mode, const Phys& P, unsigned& flags,
                                    double (&u)[S::M], double (&d)[S::Q][S::M], double& lam, double& om,
                                    bool& grad) {
  constexpr int Q = S::Q, M = S::M;
  double feq[Q][M];
  bool nz;
  node_split<S>(h, u, feq, d, nz, P);
  typename S::Node c;
  const bool adm = S::prepare(u, c, P);
  om = P.omega;
  lam = P.omega - 1.0;
  grad = false;
  if (mode == 1) {
    if (!adm) flags |= FLAG_INADMISSIBLE;
    if (!nz) {
      lam = 1.0;
    } else {
      bool fallback = !adm;
      lam = adm ? entropic_lambda<S>(c, RegSrc<S>{feq, d}, u, P, fallback) : 0.0;
      if (fallback) {
        lam = 0.0;
        flags |= FLAG_FALLBACK;
      }
      grad = !fallback;
    }
    om = lam + 1.0;
  }
}

// adjoint_root with the forward pass's lambda given (recorded by the stage
// kernel that produced this pass's output from h): no root search.
template <class S>
__device__ inline void adjoint_taped(const double (&h)[S::Q][S::M], int mode, double lam_rec, const Phys& P,
                                     double (&u)[S::M], double (&d)[S::Q][S::M], double& lam, double& om,
                                     bool& grad) {
  constexpr int Q = S::Q, M = S::M;
  double feq[Q][M];
  bool nz;
  node_split<S>(h, u, feq, d, nz, P);
  om = P.omega;
  lam = P.omega - 1.0;
  grad = false;
  if (mode == 1) {
    const bool fallback = isnan(lam_rec);
    lam = fallback ? 0.0 : lam_rec;
    grad = !fallback && nz;
    om = lam + 1.0;
  }
}

template <class S>
__device__ inline void adjoint_apply(const double (&u)[S::M], const double (&d)[S::Q][S::M], double lam, double om,
                                     bool grad, double (&gb)[S::Q][S::M], const Phys& P) {
  constexpr int Q = S::Q, M = S::M;
  typename S::Node c;
  (void)S::prepare(u, c, P);
  double feq[Q][M];
  Eq<S>::equilibrium(u, feq, P);
  double JTg[M];
  eq_jacobian_T<S>(c, gb, JTg, P);
  if (grad) {
    double dvm[Q][M], JTdv[M];
    dv_all<S>(c, feq, d, -lam, dvm, P);
    double Fp = 0.0, cc = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < M; ++m) {
        Fp += dvm[k][m] * d[k][m];
        cc -= d[k][m] * gb[k][m];
      }
    eq_jacobian_T<S>(c, dvm, JTdv, P);
    const double ratio = cc / Fp;
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < M; ++m)
        gb[k][m] = (1.0 - om) * gb[k][m] + om * JTg[m] + ((1.0 - om) * dvm[k][m] + om * JTdv[m]) * ratio;
    // the -dv(1) ratio term, one velocity at a time (dvm is dead here)
    sub_dv<S>(c, feq, d, 1.0, ratio, gb, P);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
      for (int m = 0; m < M; ++m) gb[k][m] = (1.0 - om) * gb[k][m] + om * JTg[m];
  }
}

}  // namespace eslb
