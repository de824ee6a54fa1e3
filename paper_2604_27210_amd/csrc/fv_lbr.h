// fv_lbr.h -- per-lane implied-volatility solvers in normalised coordinates.
//
// The paper (section 2.2, "Dual-Solver Design") ships two solvers behind one
// API, sharing pre- and post-processing:
//  * the "Let's Be Rational" path: boundary points of the normalised Black
//    function, a four-region rational initial guess and Householder(3)
//    steps on a three-branch transformed objective;
//  * the Halley path: a fixed number of Halley steps on the direct residual
//    and a bisection fallback for the quotes that fail a convergence check.
//    The paper starts it from the Brenner-Subrahmanyam at-the-money form;
//    here it starts from the LBR path's initial guess (that form remains
//    the fallback start), which cuts the steps a wave runs from about six
//    to three on wide-wing batches.
// Both work on the reduced problem "out-of-the-money call, x <= 0,
// 0 < beta < b_max = e^{x/2}" and return the total volatility s = sigma
// sqrt(T).
#pragma once

#include "fv_math.h"

namespace fv {

// ------------------------------------------------------- rational cubic
// Delbourgo & Gregory (SIAM J. Sci. Stat. Comput. 6(4), 1985) rational
// cubic through (xl, yl), (xr, yr) with end slopes dl, dr and control
// parameter r (r = 3 is the cubic Hermite interpolant):
//   y(tau) = [yr tau^3 + (r yr - D dr) tau^2 w + (r yl + D dl) tau w^2 + yl w^3]
//            / [1 + (r - 3) tau w],   tau = (x - xl)/D, w = 1 - tau, D = xr - xl.
__host__ __device__ inline double rational_cubic(double x, double xl, double xr, double yl,
                                                 double yr, double dl, double dr, double r) {
  const double D = xr - xl;
  if (!(D > 0.0)) return 0.5 * (yl + yr);
  double tau = (x - xl) * rcp_lo_safe(D);  // D may be denormal for deep wings
  tau = fmin(fmax(tau, 0.0), 1.0);
  const double w = 1.0 - tau;
  const double num = yr * tau * tau * tau + (r * yr - D * dr) * tau * tau * w +
                     (r * yl + D * dl) * tau * w * w + yl * w * w * w;
  const double den = 1.0 + (r - 3.0) * tau * w;
  return fdiv_lo(num, den);
}

// Smallest control parameter that keeps the interpolant monotone
// (r >= (dl + dr)/S) and convex or concave (r >= |dr - dl| / min(|dr - S|,
// |S - dl|)) when the data are; S is the secant slope.  The denominator
// stays positive for r > -1.
__host__ __device__ inline double rational_cubic_min_r(double dl, double dr, double S) {
  const double rmin = -1.0 + 1e-12;
  double r = rmin;
  const bool mono = (dl * S >= 0.0) && (dr * S >= 0.0);
  if (mono && S != 0.0) r = fmax(r, fdiv_lo(dl + dr, S));
  const bool convex = (dl <= S) && (S <= dr);
  const bool concave = (dl >= S) && (S >= dr);
  if (convex || concave) {
    const double gap = fmin(fabs(dr - S), fabs(S - dl));
    if (gap > 0.0) r = fmax(r, fdiv_lo(fabs(dr - dl), gap));
    else r = fmax(r, 1.0 / kEps);  // degenerate: fall back to (near) linear
  }
  return r;
}

// Control parameter that reproduces a given second derivative c2 at the
// left (x = xl) or right (x = xr) end:
//   y''(xl) = (2/D) [r (S - dl) + dl - dr],   y''(xr) = (2/D) [r (dr - S) + dl - dr].
__host__ __device__ inline double rational_cubic_r_left(double D, double S, double dl,
                                                        double dr, double c2) {
  return fdiv_lo(0.5 * D * c2 + dr - dl, S - dl);
}
__host__ __device__ inline double rational_cubic_r_right(double D, double S, double dl,
                                                         double dr, double c2) {
  return fdiv_lo(0.5 * D * c2 + dr - dl, dr - S);
}

__host__ __device__ inline double rational_cubic_fit(double x, double xl, double xr,
                                                     double yl, double yr, double dl,
                                                     double dr, double c2, bool fit_left) {
  const double D = xr - xl;
  const double S = (yr - yl) * rcp_lo_safe(D);
  double r = fit_left ? rational_cubic_r_left(D, S, dl, dr, c2)
                      : rational_cubic_r_right(D, S, dl, dr, c2);
  const double rmin = rational_cubic_min_r(dl, dr, S);
  if (!(r >= rmin)) r = rmin;  // also replaces NaN
  r = fmin(r, 1.0 / kEps);
  return rational_cubic(x, xl, xr, yl, yr, dl, dr, r);
}

// ------------------------------------------------------- LBR
enum Objective : int { kObjLower = 0, kObjMiddle = 1, kObjUpper = 2 };

struct LbrResult {
  double s;
  int iterations;
  bool converged;
};

// One Householder(3) step on the objective selected by `obj`, from the
// evaluation nb at s.  The three objectives of the method:
//   lower  g = 1/ln b - 1/ln beta,
//   middle g = b - beta,
//   upper  g = ln((b_max - beta)/(b_max - b)).
// nu = -g/g', eta2 = g''/g', eta3 = g'''/g' are written through
// lambda = b'/b (lower) or mu = b'/(b_max - b) (upper), eta = b''/b' and
// eta3b = b'''/b'; step = nu (1 + eta2 nu/2) / (1 + nu (eta2 + eta3 nu/6)).
template <bool LO>
__host__ __device__ inline double householder3_step_t(int obj, double x, double s, double beta,
                                                       double inv_ln_beta, double ln_bmax_m_beta,
                                                       const NBlack& nb) {
  const double is = nb.is;
  const double x2is2 = x * x * is * is;
  const double eta = x2is2 * is - 0.25 * s;                       // b''/b'
  const double eta3b = eta * eta - 3.0 * x2is2 * is * is - 0.25;  // b'''/b'
  double nu, e2, e3;
  if (obj == kObjMiddle) {
    nu = fdiv_lo(beta - nb.b, nb.bp);
    e2 = eta;
    e3 = eta3b;
  } else {
    // lower and upper share one log and one division, and both work in
    // logarithms through ratios to b', which stay in the normal range where
    // b, b_max - b and b' themselves underflow deep in the wings:
    //   lower  ln b          = ln b' + ln(b/b'),          lambda = 1/(b/b'),
    //   upper  ln(b_max - b) = ln b' + ln((b_max - b)/b'), mu    = 1/((b_max - b)/b'),
    // with (b_max - b)/b' from the complement form's E-free sum; in the
    // difference form b_max - b is taken as it is.
    const bool lo = obj == kObjLower;
    const bool comp = nb.form == kFormComplement;
    const bool plain = !lo && !comp;
    const double iw = lo ? nb.ratio : (comp ? nb.cratio : nb.c * rcp_lo_safe(nb.bp));
    const double w = LO ? rcp_lo(iw) : rcp(iw);  // lambda or mu
    const double la = plain ? nb.c : iw;
    const double lnd = (LO ? flog_lo(la) : flog(la)) + (plain ? 0.0 : nb.lnbp);
    const double L = lo ? lnd : ln_bmax_m_beta - lnd;
    if (lo) {
      const double iL = rcp_lo(L);
      nu = L * (1.0 - L * inv_ln_beta) * iw;
      e2 = eta - w * (1.0 + 2.0 * iL);
      e3 = eta3b - 3.0 * w * eta + 2.0 * w * w - 6.0 * w * (eta - w) * iL + 6.0 * w * w * iL * iL;
    } else {
      nu = -L * iw;
      e2 = eta + w;
      e3 = eta3b + 3.0 * w * eta + 2.0 * w * w;
    }
  }
  // A step that is not a number (an evaluation beyond the binary64 range)
  // becomes a halving (fmax ignores NaN); an infinite one leaves s infinite
  // and the solve unconverged.
  const double ds = fdiv_lo(nu * (1.0 + 0.5 * e2 * nu), 1.0 + nu * (e2 + e3 * nu * (1.0 / 6.0)));
  return fmax(ds, -0.5 * s);
}

__host__ __device__ inline double householder3_step(int obj, double x, double s, double beta,
                                                     double inv_ln_beta, double ln_bmax_m_beta,
                                                     const NBlack& nb) {
  return householder3_step_t<false>(obj, x, s, beta, inv_ln_beta, ln_bmax_m_beta, nb);
}

// Initial guess of the four-region scheme.  Boundary points: the inflection
// point s_c = sqrt(2|x|) of b(s), and the points s_l, s_u where the tangent
// at s_c meets 0 and b_max.  Regions in beta:
//   R1  beta < b_l          rational cubic of the lower map
//                           f_l(s) = (2 pi |x| / (3 sqrt3)) Phi(-|x|/(sqrt3 s))^3
//                           (f_l/b -> 1 as s -> 0), then f_l^{-1};
//   R2  b_l <= beta < b_c   rational cubic of s(beta), zero curvature at b_c;
//   R3  b_c <= beta <= b_u  rational cubic of s(beta), zero curvature at b_c;
//   R4  beta > b_u          rational cubic of the upper map f_u(s) = Phi(-s/2),
//                           slope -1/2 at b_max, then s = -2 Phi^{-1}(f).
// Returns s0 and sets the objective region of the iteration.
// `trace` (may be NULL) receives the path taken: bits 0-1 the guess region
// (0..3 for R1..R4), bits 4-5 and 6-7 the evaluation forms at s_c and s_o.
__host__ __device__ __attribute__((always_inline)) inline double lbr_initial_guess(
    double x, double beta, double bmax, double ln_beta, int* obj, uint32_t* trace) {
  const double ax = -x;  // |x|, x <= 0
  // At the inflection point h = -t, so b(s_c) needs one erfcx and no exp:
  //   b_c = (b_max/2) (1 - erfcx(a)),  b'(s_c) = b_max/sqrt(2 pi),  a = sqrt|x|,
  // and the lower tangent point is s_l = s_c - b_c/b'(s_c)
  //   = sqrt2 a - sqrt(pi/2) (1 - erfcx(a)).
  // Near the money both differences cancel: s_l ~ sqrt(pi/2) |x| while s_c
  // and the erfcx error are ~sqrt|x| and ~1e-8, so below a = 0.03 both come
  // from the series erfcx(a) = sum_n (-a)^n / Gamma(n/2 + 1), whose first two
  // terms cancel exactly in s_l (truncation after a^7: < a^6/24 relative).
  const double sax = sqrt_lo(ax);
  const double sc = kSqrt2 * sax;
  double om = 1.0 - erfcx_g(sax);         // 1 - erfcx(a)
  double sl = sc - kSqrtPiOver2 * om;     // s_l
  if (sax < 0.03) {
    constexpr double c3 = 4.0 / (3.0 * kSqrtPi), c5 = 8.0 / (15.0 * kSqrtPi),
                     c7 = 16.0 / (105.0 * kSqrtPi);
    // tail = 1 - c3 a + a^2/2 - c5 a^3 + a^4/6 - c7 a^5
    const double tail =
        fma(-sax, fma(-sax, fma(-sax, fma(-sax, fma(-sax, c7, 1.0 / 6.0), c5), 0.5), c3), 1.0);
    om = sax * fma(-sax, tail, kTwoOverSqrtPi);  // 2a/sqrt(pi) - a^2 tail
    sl = kSqrtPiOver2 * ax * tail;
  }
  NBlack nc;
  nc.b = 0.5 * bmax * om;
  nc.c = bmax - nc.b;
  nc.bp = kInvSqrt2Pi * bmax;
  nc.form = kFormDifference;
  const bool lower_half = beta < nc.b;
  // the other boundary point on the side of beta
  const double ibc = rcp_lo_safe(nc.bp);  // b' may underflow to 0
  const double so = lower_half ? fmax(sl, 0.0) : sc + nc.c * ibc;
  const NBlack no = normalised_black_t<2>(x, so, bmax);
  const double ibo = rcp_lo_safe(no.bp);

  const bool r1 = lower_half && beta < no.b;
  const bool r4 = !lower_half && beta > no.b;
  const bool wing = r1 || r4;
  *obj = r1 ? kObjLower : (r4 ? kObjUpper : kObjMiddle);
  if (trace)
    *trace = (uint32_t)(r1 ? 0 : (lower_half ? 1 : (r4 ? 3 : 2))) | ((uint32_t)nc.form << 4) |
             ((uint32_t)no.form << 6);

  // End data of the one rational cubic every lane evaluates.
  // R2: s(beta) on [b_l, b_c], slopes 1/b', zero curvature at b_c (b'' = 0
  //     at the inflection point): fit at the right end.
  // R3: s(beta) on [b_c, b_u], same, fit at the left end.
  double xl, xr, yl, yr, dl, dr, c2 = 0.0;
  bool fit_left = !lower_half;
  if (lower_half) {
    xl = no.b; xr = nc.b; yl = so; yr = sc; dl = ibo; dr = ibc;
  } else {
    xl = nc.b; xr = no.b; yl = sc; yr = so; dl = ibc; dr = ibo;
  }
  const double cl = ax * (2.0 * kPi / (3.0 * kSqrt3));  // 2 pi |x| / (3 sqrt3)
  if (wing) {
    // R1 / R4 share one Phi/phi evaluation at the transformed boundary point
    // (lower map: z = -|x|/(sqrt3 s_l); upper map: z = -s_u/2).  With
    // b''/b' = eta:  df/dbeta = f'/b',  d2f/dbeta2 = (f'' - f' eta)/b'^2.
    const double iso = rcp_lo(so);
    const double eta_o = x * x * iso * iso * iso - 0.25 * so;  // b''/b' at s_o
    const double z = r1 ? -ax * (1.0 / kSqrt3) * iso : -0.5 * so;
    const double ez = fexp_g(-0.5 * z * z);
    const double Pz = 0.5 * ez * erfcx_g(-z * kInvSqrt2);   // Phi(z), z <= 0
    const double pz = kInvSqrt2Pi * ez;                          // phi(z)
    double f0, f1, f2;  // f, df/ds, d2f/ds2 at s_o
    if (r1) {
      const double zp = -z * iso;  // dz/ds
      f0 = cl * Pz * Pz * Pz;
      f1 = 3.0 * cl * Pz * Pz * pz * zp;
      // d2f/ds2 = 3 cl z'^2 Phi phi (2 phi - Phi z + 2 Phi/z); with
      // z = -|x|/(sqrt3 s) the last term times cl is -(4 pi/3) Phi s_o, so
      // no division is needed
      f2 = 3.0 * zp * zp * Pz * pz * fma(cl, fma(-Pz, z, 2.0 * pz), -(4.0 * kPi / 3.0) * Pz * so);
    } else {
      f0 = Pz;
      f1 = -0.5 * pz;
      f2 = 0.125 * so * pz;
    }
    const double dfo = f1 * ibo;
    const double c2o = (f2 - f1 * eta_o) * ibo * ibo;
    if (r1) {
      // f on [0, b_l]: (0, 0) slope 1 -> (b_l, f_l(s_l)) slope dfo; fit right
      xl = 0.0; xr = no.b; yl = 0.0; yr = f0; dl = 1.0; dr = dfo; c2 = c2o; fit_left = false;
    } else {
      // f on [b_u, b_max]: (b_u, f_u(s_u)) slope dfo, fit left -> (b_max, 0) slope -1/2
      xl = no.b; xr = bmax; yl = f0; yr = 0.0; dl = dfo; dr = -0.5; c2 = c2o; fit_left = true;
    }
  }
  const double y = rational_cubic_fit(beta, xl, xr, yl, yr, dl, dr, c2, fit_left);
  if (!wing) return y;
  // invert the map: R1 Phi(z) = (f/cl)^{1/3}, s = -|x|/(sqrt3 z);
  //                 R4 Phi(-s/2) = f,          s = -2 z.
  // The inverse normal needs only ln p: R1 ln p = ln(f/cl)/3, R4 ln p = ln f,
  // one logarithm either way.  The lower-map cubic leaves (0, 0) with slope
  // 1, so for a beta below the normal range f = beta (1 + O(beta)): there
  // ln(f/cl) is taken as ln beta - ln cl, which stays finite where f
  // underflows.
  const double f = fmax(y, 1e-300);
  const bool deep = r1 && y < 0x1p-960;
  const double la = flog_lo(r1 ? (deep ? cl : f * rcp_lo(cl)) : fmin(f, 0.5));
  const double lnp = r1 ? fmin((deep ? ln_beta - la : la) * (1.0 / 3.0),
                               -0.69314718076)  // p <= 0.4999999999
                        : la;
  const double zi = inv_norm_cdf_lower_ln_g(lnp);
  return r1 ? -ax * (1.0 / kSqrt3) * rcp_lo(zi) : -2.0 * zi;
}

// Full LBR solve: guess, then Householder(3) steps.  `min_steps` steps are
// always taken; more (up to `max_steps`) while the last step exceeds
// `step_tol` relative -- on the GPU this makes the extra step a wave-level
// decision, taken only by waves holding a lane that needs it.
// `trace` (may be NULL) receives the guess path (see lbr_initial_guess),
// bits 2-3 the number of steps minus 2 and, from bit 8, two bits per step
// for the evaluation form of that step.
__host__ __device__ __attribute__((always_inline)) inline LbrResult lbr_solve(
    double x, double beta, double bmax, double ln_beta, int min_steps, int max_steps,
    double step_tol, uint32_t* trace = nullptr) {
  int obj;
  double s = lbr_initial_guess(x, beta, bmax, ln_beta, &obj, trace);
  const double inv_ln_beta = rcp(ln_beta);
  // ln(b_max - beta), the upper objective's target, once per quote
  double ln_bmax_m_beta = 0.0;
  if (obj == kObjUpper) ln_bmax_m_beta = flog(bmax - beta);
  LbrResult res;
  // The first step starts ~1e-2 from the root and lands ~1e-8 from it, so it
  // runs at guess precision (b to ~1e-8); every later step is at full
  // precision and decides the converged root.
  int it = 0;
  double ds = 0.0;
  if (max_steps > 0) {
    const NBlack nb = normalised_black_t<1>(x, s, bmax);
    if (trace) *trace |= (uint32_t)nb.form << 8;
    ds = householder3_step_t<true>(obj, x, s, beta, inv_ln_beta, ln_bmax_m_beta, nb);
    s += ds;
    it = 1;
  }
  for (; it < max_steps; ++it) {
    if (it >= min_steps && !(fabs(ds) > step_tol * s)) break;
    const NBlack nb = normalised_black(x, s, bmax);
    if (trace) *trace |= (uint32_t)nb.form << (8 + 2 * it);
    ds = householder3_step(obj, x, s, beta, inv_ln_beta, ln_bmax_m_beta, nb);
    s += ds;
  }
  if (trace) *trace |= (uint32_t)(it - 2) << 2;
  res.s = s;
  res.iterations = it;
  // converged: the loop stopped on the step test (or the last step passed
  // it) at a finite positive root
  res.converged = (!(fabs(ds) > step_tol * s) || it < max_steps) && s > 0.0 && __builtin_isfinite(s);
  return res;
}

// ------------------------------------------------------- Halley path
struct HalleyState {
  double s, lo, hi;
  int steps;  // Halley steps taken
  bool converged;
};

// Normalised prices below this (2^-960) are solved on the logarithmic
// residual ln b(s) - ln beta: there beta, and b near the root, are at or
// below the edge of the normal binary64 range, keep few significant bits,
// and the direct residual b - beta and its relative test lose their meaning.
constexpr double kLnBetaLogResidual = -665.4;  // ln 2^-960

// ln b(x, s) from an evaluation: ln b' + ln(b/b') in the difference form
// (both parts stay in the normal range however small b is), ln b in the
// complement form (where b >= 0.3 b_max).
__host__ __device__ inline double ln_nb(const NBlack& nb) {
  return nb.form == kFormDifference ? nb.lnbp + flog(nb.ratio) : flog(nb.b);
}

// One Halley step from s; `res` receives the residual at s and `st` the
// bracket its sign fixes.  Two residuals:
//  * direct (beta >= 2^-960): g = b(s) - beta, step = nu/(1 + eta nu/2),
//    nu = -g/b', eta = b''/b';
//  * logarithmic (beta < 2^-960): g = ln b(s) - ln beta, g' = b'/b = lambda,
//    g''/g' = eta - lambda, step = nu/(1 + (eta - lambda) nu/2), nu = -g/lambda.
// Safeguards (the paper does not spell its own out):
//  * far below the root of an out-of-the-money quote b(s) behaves like
//    C s^3 exp(-x^2/(2 s^2)), so on the direct residual the curvature term
//    makes the Halley step crawl (step ~ 2 s^3/x^2).  When the residual is
//    negative and the Halley factor 1/(1 + eta nu/2) has dropped below 1/2,
//    the step is a Newton step on ln b - ln beta in u = 1/s^2, where ln b is
//    nearly linear (or, when b underflowed, to max(2 s, |x|/sqrt(-2 ln beta)),
//    the root of the leading-order form);
//  * a bracket [lo, hi] from the sign of the residual keeps every iterate
//    inside; a step that would leave it bisects instead (geometrically).
// P is the evaluation's precision level (normalised_black_t).  Only a
// full-precision residual (P = 0) moves the bracket: near the root the
// sign of a guess-precision residual is not reliable.
template <int P>
__host__ __device__ __attribute__((always_inline)) inline double halley_step_t(
    double x, double beta, double bmax, double ln_beta, bool logres, double s, HalleyState& st,
    double& res) {
  const NBlack nb = normalised_black_t<P>(x, s, bmax);
  const double is0 = nb.is;
  const double eta = x * x * is0 * is0 * is0 - 0.25 * s;  // b''/b'
  double sn;
  if (logres) {
    res = ln_nb(nb) - ln_beta;
    if (P == 0) {
      if (res < 0.0) st.lo = s; else st.hi = s;
    }
    const double lam = rcp(nb.ratio);  // b'/b
    const double nu = -res * nb.ratio;
    sn = s + nu * rcp_lo(1.0 + 0.5 * (eta - lam) * nu);
  } else {
    res = nb.b - beta;
    if (P == 0) {
      if (res < 0.0) st.lo = s; else st.hi = s;
    }
    const double nu = -res * rcp(nb.bp);
    const double hf = rcp_lo(1.0 + 0.5 * eta * nu);
    sn = s + nu * hf;
    if (res < 0.0 && !(hf >= 0.5) && x < 0.0) {
      // Newton step on ln b - ln beta in u = 1/s^2, where ln b is close to
      // linear: d ln b/du = -(b'/b) s^3/2.  If b underflowed (to zero or a
      // denormal) or the step is unusable, the root of the leading-order form
      // b ~ exp(-x^2/(2 s^2)), but at least 2 s.
      double un = -1.0;
      if (nb.b > 1e-290) {
        const double dLdu = -0.5 * nb.bp * rcp_lo(nb.b) * s * s * s;
        un = fma(fdiv_lo(ln_beta - flog(nb.b), dLdu), 1.0, is0 * is0);
      }
      sn = (un > 0.0 && un < 1e300) ? rsqrt(un) : fmax(2.0 * s, -x * rsqrt(-2.0 * ln_beta));
    }
  }
  // inclusive test: at the root the step rounds to 0 and s is a bound
  if (!(sn >= st.lo && sn <= st.hi)) {
    if (st.hi >= 1e300) sn = 2.0 * s + 1e-3;
    else if (st.lo > 0.0) sn = sqrt(st.lo) * sqrt(st.hi);  // no underflow of lo hi
    else sn = 0.5 * st.hi;
  }
  return sn;
}

// Start: the four-region initial guess of the LBR path (a few percent from
// the root at worst), or, where it is not a positive finite number, the
// larger of the Brenner-Subrahmanyam at-the-money form s0 = sqrt(2 pi) beta
// and the root |x|/sqrt(-2 ln beta) of the leading-order wing form
// ln b ~ -x^2/(2 s^2).  Then at most `steps` Halley steps, the first at
// guess precision (from ~1e-2 it lands ~1e-6 from the root, far above that
// evaluation's error), every later one at full precision.  Halley converges
// cubically: after a step below 1e-5 s the error left is about
// kc (1e-5)^3 s, where the error constant kc = (eta s)^2/12 + h^2/2 +
// s^2/24 is up to about 130 on the wide workload (|h| <= 6), and below
// 1e-8 s up to |h| of about 100 (beyond |h| ~ 37 the root is solved on the
// nearly linear logarithmic residual).  So a lane stops at the first full-
// precision step below 1e-5 s (a wave whose lanes have all stopped leaves
// the loop early).  Converged: that stop, the residual before the last step
// within 1e-2 relative (a sanity check against a stall where b' vanishes;
// near the root the residual is the step times s b'/b, at most 1e-5 h^2),
// and a positive finite s.
constexpr double kHalleyStepTol = 1e-5;

__host__ __device__ __attribute__((always_inline)) inline HalleyState halley_solve(
    double x, double beta, double bmax, double ln_beta, int steps) {
  HalleyState st;
  st.lo = 0.0;
  st.hi = 1e300;
  const bool logres = ln_beta < kLnBetaLogResidual;
  int region;
  double s = lbr_initial_guess(x, beta, bmax, ln_beta, &region, nullptr);
  // the guess-precision first step only from the guess (whose |h| is
  // bounded); from the fallback start every step is at full precision
  const bool from_guess = s > 0.0 && s < 1e300;
  if (!from_guess) {
    const double s_bs = kSqrt2Pi * beta;
    s = x < 0.0 ? fmax(s_bs, -x * rsqrt(-2.0 * ln_beta)) : s_bs;
  }
  double ds = 0.0, res = 0.0;
  bool stop = false;
  int k = 0;
  if (from_guess && steps > 0) {
    const double sn = halley_step_t<1>(x, beta, bmax, ln_beta, logres, s, st, res);
    ds = sn - s;
    s = sn;
    k = 1;
  }
  while (k < steps) {
    const double sn = halley_step_t<0>(x, beta, bmax, ln_beta, logres, s, st, res);
    ds = sn - s;
    s = sn;
    ++k;
    stop = fabs(ds) <= kHalleyStepTol * s;
    if (stop) break;
  }
  st.s = s;
  st.steps = k;
  st.converged = stop && fabs(res) <= (logres ? 1e-2 : 1e-2 * beta) && s > 0.0 &&
                 __builtin_isfinite(s);
  return st;
}

// Bisection on ln s inside [lo, hi] to rel_tol, comparing b with beta (in
// logarithms below 2^-960, as the Halley residual does).
__host__ __device__ inline double bisection_solve(double x, double beta, double bmax,
                                                  double ln_beta, double lo, double hi,
                                                  double rel_tol) {
  // an end the caller's bracket did not fix: far below any root, and far
  // above it (b_max - b(s) < b_max 1e-16 once s exceeds ~20 + |x|/10)
  if (!(lo > 0.0)) lo = 1e-300;
  if (!(hi < 1e300)) hi = 1e3;
  const bool logres = ln_beta < kLnBetaLogResidual;
  // geometric midpoints as sqrt(lo) sqrt(hi): lo hi may underflow
  for (int k = 0; k < 200 && hi - lo > rel_tol * hi; ++k) {
    const double mid = sqrt(lo) * sqrt(hi);
    const NBlack nb = normalised_black(x, mid, bmax);
    const bool below = logres ? ln_nb(nb) < ln_beta : nb.b < beta;
    if (below) lo = mid; else hi = mid;
  }
  return sqrt(lo) * sqrt(hi);
}

}  // namespace fv
