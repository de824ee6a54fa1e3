// fv_lbr.h -- per-lane implied-volatility solvers in normalised coordinates.
//
// The paper (section 2.2, "Dual-Solver Design") ships two solvers behind one
// API, sharing pre- and post-processing:
//  * the "Let's Be Rational" path: boundary points of the normalised Black
//    function, a four-region rational initial guess and Householder(3)
//    steps on a three-branch transformed objective;
//  * the Halley path: a Brenner-Subrahmanyam at-the-money start, a fixed
//    number of Halley steps on the direct residual and a bisection fallback
//    for the quotes that fail a convergence check.
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
  double tau = (x - xl) / D;
  tau = fmin(fmax(tau, 0.0), 1.0);
  const double w = 1.0 - tau;
  const double num = yr * tau * tau * tau + (r * yr - D * dr) * tau * tau * w +
                     (r * yl + D * dl) * tau * w * w + yl * w * w * w;
  const double den = 1.0 + (r - 3.0) * tau * w;
  return num / den;
}

// Smallest control parameter that keeps the interpolant monotone
// (r >= (dl + dr)/S) and convex or concave (r >= |dr - dl| / min(|dr - S|,
// |S - dl|)) when the data are; S is the secant slope.  The denominator
// stays positive for r > -1.
__host__ __device__ inline double rational_cubic_min_r(double dl, double dr, double S) {
  const double rmin = -1.0 + 1e-12;
  double r = rmin;
  const bool mono = (dl * S >= 0.0) && (dr * S >= 0.0);
  if (mono && S != 0.0) r = fmax(r, (dl + dr) / S);
  const bool convex = (dl <= S) && (S <= dr);
  const bool concave = (dl >= S) && (S >= dr);
  if (convex || concave) {
    const double gap = fmin(fabs(dr - S), fabs(S - dl));
    if (gap > 0.0) r = fmax(r, fabs(dr - dl) / gap);
    else r = fmax(r, 1.0 / kEps);  // degenerate: fall back to (near) linear
  }
  return r;
}

// Control parameter that reproduces a given second derivative c2 at the
// left (x = xl) or right (x = xr) end:
//   y''(xl) = (2/D) [r (S - dl) + dl - dr],   y''(xr) = (2/D) [r (dr - S) + dl - dr].
__host__ __device__ inline double rational_cubic_r_left(double D, double S, double dl,
                                                        double dr, double c2) {
  return (0.5 * D * c2 + dr - dl) / (S - dl);
}
__host__ __device__ inline double rational_cubic_r_right(double D, double S, double dl,
                                                         double dr, double c2) {
  return (0.5 * D * c2 + dr - dl) / (dr - S);
}

__host__ __device__ inline double rational_cubic_fit(double x, double xl, double xr,
                                                     double yl, double yr, double dl,
                                                     double dr, double c2, bool fit_left) {
  const double D = xr - xl;
  const double S = (yr - yl) / D;
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
__host__ __device__ inline double householder3_step(int obj, double x, double s, double beta,
                                                     double ln_beta, double bmax,
                                                     const NBlack& nb) {
  const double eta = nb_d2_over_d1(x, s);
  const double eta3b = nb_d3_over_d1(x, s, eta);
  double nu, e2, e3;
  if (obj == kObjLower) {
    const double L = log(nb.b);
    const double lam = nb.bp / nb.b;
    const double iL = 1.0 / L;
    nu = L * (ln_beta - L) / (lam * ln_beta);
    e2 = eta - lam * (1.0 + 2.0 * iL);
    e3 = eta3b - 3.0 * lam * eta + 2.0 * lam * lam - 6.0 * lam * (eta - lam) * iL +
         6.0 * lam * lam * iL * iL;
  } else if (obj == kObjUpper) {
    const double mu = nb.bp / nb.c;
    nu = -log((bmax - beta) / nb.c) / mu;
    e2 = eta + mu;
    e3 = eta3b + 3.0 * mu * eta + 2.0 * mu * mu;
  } else {
    nu = (beta - nb.b) / nb.bp;
    e2 = eta;
    e3 = eta3b;
  }
  double ds = nu * (1.0 + 0.5 * e2 * nu) / (1.0 + nu * (e2 + e3 * nu * (1.0 / 6.0)));
  if (!(ds == ds)) ds = 0.0;
  return fmax(ds, -0.5 * s);
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
__host__ __device__ inline double lbr_initial_guess(double x, double beta, double bmax,
                                                    int* obj) {
  const double ax = -x;  // |x|, x <= 0
  const double sc = sqrt(2.0 * ax);
  const NBlack nc = normalised_black(x, sc, bmax);
  const bool lower_half = beta < nc.b;
  // the other boundary point on the side of beta
  const double so = lower_half ? fmax(sc - nc.b / nc.bp, 0.0) : sc + nc.c / nc.bp;
  const NBlack no = normalised_black(x, so, bmax);

  const bool r1 = lower_half && beta < no.b;
  const bool r4 = !lower_half && beta > no.b;
  *obj = r1 ? kObjLower : (r4 ? kObjUpper : kObjMiddle);

  if (!(r1 || r4)) {
    // R2 / R3: interpolate s(beta) between the two boundary points; slopes
    // ds/dbeta = 1/b'.  b'' = 0 at s_c gives zero curvature at b_c.
    if (lower_half)
      return rational_cubic_fit(beta, no.b, nc.b, so, sc, 1.0 / no.bp, 1.0 / nc.bp, 0.0,
                                false);
    return rational_cubic_fit(beta, nc.b, no.b, sc, so, 1.0 / nc.bp, 1.0 / no.bp, 0.0, true);
  }

  // R1 / R4: one Phi evaluation at the transformed boundary point.
  //   f(beta) derivatives from the chain rule with b' and
  //   b''/b' = eta:  df/dbeta = f'/b',  d2f/dbeta2 = (f'' - f' eta)/b'^2.
  const double eta_o = nb_d2_over_d1(x, so);
  double guess;
  if (r1) {
    const double cl = 2.0 * kPi * ax / (3.0 * kSqrt3);
    const double z = -ax / (kSqrt3 * so);
    const double Pz = norm_cdf(z), pz = norm_pdf(z);
    const double zp = -z / so;               // dz/ds
    const double fl = cl * Pz * Pz * Pz;
    const double f1 = 3.0 * cl * Pz * Pz * pz * zp;
    const double f2 = 3.0 * cl * (2.0 * Pz * pz * pz * zp * zp - Pz * Pz * z * pz * zp * zp +
                                  Pz * Pz * pz * (-2.0 * zp / so));
    const double dr = f1 / no.bp;
    const double c2 = (f2 - f1 * eta_o) / (no.bp * no.bp);
    double f = rational_cubic_fit(beta, 0.0, no.b, 0.0, fl, 1.0, dr, c2, false);
    f = fmax(f, 1e-300);
    const double u = cbrt(f / cl);           // Phi(z) at the guess, < 1/2
    guess = -ax / (kSqrt3 * inv_norm_cdf_lower(fmin(u, 0.4999999999)));
  } else {
    const double z = -0.5 * so;
    const double fu = norm_cdf(z), pz = norm_pdf(z);
    const double f1 = -0.5 * pz;             // d f_u / ds
    const double f2 = 0.125 * so * pz;       // d2 f_u / ds2
    const double dl = f1 / no.bp;
    const double c2 = (f2 - f1 * eta_o) / (no.bp * no.bp);
    double f = rational_cubic_fit(beta, no.b, bmax, fu, 0.0, dl, -0.5, c2, true);
    f = fmin(fmax(f, 1e-300), 0.5);
    guess = -2.0 * inv_norm_cdf_lower(f);
  }
  return guess;
}

// Full LBR solve: guess, then Householder(3) steps.  `min_steps` steps are
// always taken; more (up to `max_steps`) while the last step exceeds
// `step_tol` relative -- on the GPU this makes the extra step a wave-level
// decision, taken only by waves holding a lane that needs it.
__host__ __device__ inline LbrResult lbr_solve(double x, double beta, int min_steps,
                                               int max_steps, double step_tol) {
  const double bmax = exp(0.5 * x);
  int obj;
  double s = lbr_initial_guess(x, beta, bmax, &obj);
  const double ln_beta = log(beta);
  LbrResult res;
  int it = 0;
  double ds = 0.0;
  for (; it < max_steps; ++it) {
    if (it >= min_steps && !(fabs(ds) > step_tol * s)) break;
    const NBlack nb = normalised_black(x, s, bmax);
    ds = householder3_step(obj, x, s, beta, ln_beta, bmax, nb);
    s += ds;
  }
  res.s = s;
  res.iterations = it;
  res.converged = !(fabs(ds) > step_tol * s) || it < max_steps;
  return res;
}

// ------------------------------------------------------- Halley path
struct HalleyState {
  double s, lo, hi;
  bool converged;
};

// Brenner-Subrahmanyam start s0 = sqrt(2 pi) beta (the at-the-money
// approximation b(0, s) ~ s/sqrt(2 pi)), then `steps` Halley steps on the
// direct residual b(s) - beta: step = nu/(1 + eta nu/2), nu = (beta - b)/b'.
// A bracket [lo, hi] from the sign of the residual keeps every iterate
// inside; a step that would leave it bisects instead (geometrically).
// Converged: last |step| <= 1e-10 s and |b - beta| <= 1e-9 beta.
__host__ __device__ inline HalleyState halley_solve(double x, double beta, int steps) {
  const double bmax = exp(0.5 * x);
  HalleyState st;
  st.lo = 0.0;
  st.hi = 1e300;
  double s = kSqrt2Pi * beta;
  double ds = 0.0, res = 0.0;
  for (int k = 0; k < steps; ++k) {
    const NBlack nb = normalised_black(x, s, bmax);
    res = nb.b - beta;
    if (res < 0.0) st.lo = s; else st.hi = s;
    const double nu = -res / nb.bp;
    const double eta = nb_d2_over_d1(x, s);
    double sn = s + nu / (1.0 + 0.5 * eta * nu);
    if (!(sn > st.lo && sn < st.hi)) {
      if (st.hi >= 1e300) sn = 2.0 * s + 1e-3;
      else if (st.lo > 0.0) sn = sqrt(st.lo * st.hi);
      else sn = 0.5 * st.hi;
    }
    ds = sn - s;
    s = sn;
  }
  st.s = s;
  st.converged = fabs(ds) <= 1e-10 * s && fabs(res) <= 1e-9 * beta;
  return st;
}

// Bisection on ln s inside [lo, hi] until the bracket is below `rel_tol`.
__host__ __device__ inline double bisection_solve(double x, double beta, double lo,
                                                  double hi, double rel_tol) {
  const double bmax = exp(0.5 * x);
  if (!(lo > 0.0)) lo = 1e-8;
  if (!(hi < 1e300)) hi = 50.0;
  for (int k = 0; k < 200 && hi - lo > rel_tol * hi; ++k) {
    const double mid = sqrt(lo * hi);
    const NBlack nb = normalised_black(x, mid, bmax);
    if (nb.b < beta) lo = mid; else hi = mid;
  }
  return sqrt(lo * hi);
}

}  // namespace fv
