// fv_math.h -- FP64 special functions and the normalised Black function.
//
// Everything here is __host__ __device__ and branch-light: the kernels call
// it per lane, so a data-dependent branch costs the union of its sides only
// when lanes of one wave disagree (the compiler skips a side whose exec mask
// is empty).
//
// Notation (normalised Black coordinates of the paper's section 1 and the
// "Let's Be Rational" method it cites in section 2.2):
//   x = ln(F/K), s = sigma sqrt(T), h = x/s, t = s/2,
//   b(x, s)   = e^{x/2} Phi(h + t) - e^{-x/2} Phi(h - t)   (call),
//   b_max     = e^{x/2},   price = D sqrt(F K) b.
// After the reduction to an out-of-the-money call the solvers only ever need
// x <= 0, where b rises from 0 to b_max.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_coeffs.h"

namespace fv {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kInvSqrt2 = 0.70710678118654752440;
constexpr double kSqrt2Pi = 2.50662827463100050242;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kSqrtPiOver2 = 1.25331413731550025121;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;
constexpr double kLnSqrt2Pi = 0.91893853320467274178;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kEps = 2.220446049250313e-16;
constexpr double kDblMin = 2.2250738585072014e-308;  // smallest normal binary64

// ----------------------------------------------------------- reciprocal
// 1/x for finite, normal, non-zero x: the hardware estimate v_rcp_f64
// refined by two Newton steps (r <- r + r (1 - x r)), within ~1 ulp.  Cheaper
// than an IEEE division, which also handles zero, infinite and denormal
// operands: for those the refinement yields NaN (see rcp_safe).
__host__ __device__ inline double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
#else
  return 1.0 / x;
#endif
}

// As rcp, but 1/0 = inf and 1/inf = 0 as for a division (the hardware
// estimate is exact there and is kept when the refinement turns to NaN).
__host__ __device__ inline double rcp_safe(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r0 = __builtin_amdgcn_rcp(x);
  double r = fma(r0, fma(-x, r0, 1.0), r0);
  r = fma(r, fma(-x, r, 1.0), r);
  return r == r ? r : r0;
#else
  return 1.0 / x;
#endif
}

// a/b from the refined reciprocal plus one residual correction (~1 ulp).
__host__ __device__ inline double fdiv(double a, double b) {
  const double r = rcp(b);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// 1/sqrt(x) for finite positive normal x: v_rsq_f64 refined by two Newton
// steps y <- y + y (1/2 - x y^2 / 2).
__host__ __device__ inline double rsqrt(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = fma(y, fma(-hx * y, y, 0.5), y);
  y = fma(y, fma(-hx * y, y, 0.5), y);
  return y;
#else
  return 1.0 / sqrt(x);
#endif
}

// ------------------------------------------------------------ exp / log
// Lean binary64 exp and log for the solver's finite arguments (the HIP
// library versions also handle every special input, which these call sites
// never pass, at two to three times the instruction count).
//
// exp: Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, with ln2 split in a
// high part exact in binary64 products and a low part; e^r by its Taylor
// series to degree 13 (truncation < 4e-18 on |r| <= ln2/2); 2^n by ldexp.
// Arguments below -1000 give 0 (ldexp underflows), NaN propagates.
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln2 - kLn2Hi
constexpr double kLog2E = 1.44269504088896338700e+00;

__host__ __device__ inline double fexp(double x) {
  x = x < -1000.0 ? -1000.0 : x;
  const double n = rint(x * kLog2E);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
  double p = 1.0 / 6227020800.0;                      // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);                   // 1/12!
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// log for positive finite x (0 gives -inf): x = 2^e m with m in
// [sqrt(1/2), sqrt(2)), f = (m - 1)/(m + 1), ln m = 2 atanh(f) =
// 2f (1 + f^2/3 + f^4/5 + ...), |f| <= 0.1716 so ten terms reach binary64
// precision; ln x = e ln2 + ln m with ln2 split as in fexp.
__host__ __device__ inline double flog(double x) {
  int e;
  double m = frexp(x, &e);  // m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double f = fdiv(m - 1.0, m + 1.0);  // m + 1 in [1.7, 2.5]
  const double z = f * f;
  double S = 1.0 / 21.0;
  S = fma(S, z, 1.0 / 19.0);
  S = fma(S, z, 1.0 / 17.0);
  S = fma(S, z, 1.0 / 15.0);
  S = fma(S, z, 1.0 / 13.0);
  S = fma(S, z, 1.0 / 11.0);
  S = fma(S, z, 1.0 / 9.0);
  S = fma(S, z, 1.0 / 7.0);
  S = fma(S, z, 1.0 / 5.0);
  S = fma(S, z, 1.0 / 3.0);
  const double f2 = f + f;
  const double de = (double)e;
  const double lm = fma(f2 * z, S, f2);  // 2f + 2f z S(z)
  const double res = fma(de, kLn2Hi, fma(de, kLn2Lo, lm));
  return x == 0.0 ? -__builtin_inf() : res;
}

// ------------------------------------------------ guess-precision helpers
// The initial guess of the implied-volatility iteration only has to land
// within ~1e-3 of the root (two quartically convergent steps then reach
// binary64 precision), and the Householder step itself only needs a relative
// precision well below its own size.  These variants stop at ~1e-8 relative
// (one Newton refinement, shorter series) and are used only there; every
// quantity that decides where the iteration converges -- b(s), its
// complement, ln b, ln beta -- keeps the full-precision routines.
__host__ __device__ inline double rcp_lo(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}

// rcp_lo that keeps the exact 1/0 = inf and 1/inf = 0 of the estimate
__host__ __device__ inline double rcp_lo_safe(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r0 = __builtin_amdgcn_rcp(x);
  const double r = fma(r0, fma(-x, r0, 1.0), r0);
  return r == r ? r : r0;
#else
  return 1.0 / x;
#endif
}

__host__ __device__ inline double fdiv_lo(double a, double b) { return a * rcp_lo(b); }

// sqrt(x) for x >= 0 as x / sqrt(x) from the refined reciprocal square root
__host__ __device__ inline double sqrt_lo(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(x);
  y = fma(y, fma(-0.5 * x * y, y, 0.5), y);
  return x > 0.0 ? x * y : 0.0;
#else
  return sqrt(x);
#endif
}

// e^x with the reduction of fexp and the Taylor series to degree 8
// (truncation < 2.2e-10 on |r| <= ln2/2)
__host__ __device__ inline double fexp_lo(double x) {
  x = x < -1000.0 ? -1000.0 : x;
  const double n = rint(x * kLog2E);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
  double p = 1.0 / 40320.0;
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// e^x with the reduction of fexp and the Taylor series to degree 6
// (truncation < 1.3e-7 on |r| <= ln2/2), for the initial guess only
__host__ __device__ inline double fexp_g(double x) {
  x = x < -1000.0 ? -1000.0 : x;
  const double n = rint(x * kLog2E);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
  double p = 1.0 / 720.0;
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// ln x with the reduction of flog and five terms of the atanh series
// (truncation < 7e-10 for |f| <= 0.1716)
__host__ __device__ inline double flog_lo(double x) {
  int e;
  double m = frexp(x, &e);
  if (m < 0.70710678118654752440) {
    m += m;
    --e;
  }
  const double f = fdiv_lo(m - 1.0, m + 1.0);
  const double z = f * f;
  double S = 1.0 / 9.0;
  S = fma(S, z, 1.0 / 7.0);
  S = fma(S, z, 1.0 / 5.0);
  S = fma(S, z, 1.0 / 3.0);
  const double f2 = f + f;
  const double de = (double)e;
  const double res = fma(de, kLn2Hi, fma(f2 * z, S, f2));
  return x == 0.0 ? -__builtin_inf() : res;
}

// ----------------------------------------------------------------- erfcx
// erfcx(z) = exp(z^2) erfc(z) for z >= -Z0 (Z0 = 1/2), one branch-free
// polynomial p in y = (z - B + 2 Z0)/(z + B): erfcx(z) = p(y)/(z + B)
// (fitted coefficients, fv_coeffs.h).
constexpr int kErfcxDeg = (int)(sizeof(coef::kErfcx) / sizeof(double)) - 1;

__host__ __device__ inline double erfcx_fit(double z) {
  const double R = rcp(z + coef::kErfcxB);
  const double y = (z - (coef::kErfcxB - 2.0 * coef::kErfcxZ0)) * R;
  double p = coef::kErfcx[kErfcxDeg];
#pragma unroll
  for (int i = kErfcxDeg - 1; i >= 0; --i) p = fma(p, y, coef::kErfcx[i]);
  return p * R;
}

// Degree of the first Householder step's fit (relative error ~1e-8).
constexpr int kErfcxLoDeg = (int)(sizeof(coef::kErfcxLo) / sizeof(double)) - 1;

// The same form with the initial guess's fit (degree 7, relative error
// ~4e-6): the guess lands a few percent from the root, far above that.
constexpr int kErfcxGDeg = (int)(sizeof(coef::kErfcxG) / sizeof(double)) - 1;

__host__ __device__ inline double erfcx_g(double z) {
  const double R = rcp_lo(z + coef::kErfcxGB);
  const double y = (z - (coef::kErfcxGB - 2.0 * coef::kErfcxZ0)) * R;
  double p = coef::kErfcxG[kErfcxGDeg];
#pragma unroll
  for (int i = kErfcxGDeg - 1; i >= 0; --i) p = fma(p, y, coef::kErfcxG[i]);
  return p * R;
}

// Standard normal density and CDF.  Phi goes through erfcx so that the lower
// tail keeps full relative precision (paper section 2.3 evaluates the CDF
// through the complementary error function for the same reason).
__host__ __device__ inline double norm_pdf(double z) { return kInvSqrt2Pi * fexp(-0.5 * z * z); }

__host__ __device__ inline double norm_cdf(double z) {
  const double a = fabs(z) * kInvSqrt2;
  const double tail = 0.5 * fexp(-0.5 * z * z) * erfcx_fit(a);  // Phi(-|z|)
  return z < 0.0 ? tail : 1.0 - tail;
}

// Inverse standard normal CDF for p in (0, 1/2] (returns a value <= 0), from
// ln p alone: (r - r0) P(r)/Q(r) with r = sqrt(-2 ln p) and r0 = sqrt(2 ln 2)
// (r at p = 1/2, where the inverse has its simple zero), one [3/3] rational
// on the whole range, relative error ~2e-6 (fitted, fv_coeffs.h).  Only the
// initial guess uses it; ln p stays finite where p itself underflows.
constexpr int kPhiInvGDegP = (int)(sizeof(coef::kPhiInvGP) / sizeof(double)) - 1;
constexpr int kPhiInvGDegQ = (int)(sizeof(coef::kPhiInvGQ) / sizeof(double)) - 1;

__host__ __device__ inline double inv_norm_cdf_lower_ln_g(double lnp) {
  const double r = sqrt_lo(-2.0 * lnp);
  double num = coef::kPhiInvGP[kPhiInvGDegP], den = coef::kPhiInvGQ[kPhiInvGDegQ];
#pragma unroll
  for (int i = kPhiInvGDegP - 1; i >= 0; --i) num = fma(num, r, coef::kPhiInvGP[i]);
#pragma unroll
  for (int i = kPhiInvGDegQ - 1; i >= 0; --i) den = fma(den, r, coef::kPhiInvGQ[i]);
  return (r - coef::kPhiInvGR0) * fdiv_lo(num, den);
}

// ---------------------------------------------------- normalised Black
// With q1 = -(h+t)/sqrt2, q2 = (t-h)/sqrt2 >= |q1| (x <= 0) and
// E = exp(-(h^2+t^2)/2):
//     b       = E/2 [erfcx(q1) - erfcx(q2)],
//     b_max-b = E/2 [erfcx(-q1) + erfcx(q2)],
//     b'      = db/ds = E/sqrt(2 pi).
// One evaluation form serves every (x, s), so a wave never splits:
//
//  * difference form (q1 >= -Z0): the two erfcx values come from the same
//    polynomial p, so their difference is taken as a divided difference,
//    never by subtraction.  With R_i = 1/(q_i + B), y_i = p's abscissae,
//        erfcx(q1) - erfcx(q2) = R1 (p(y1) - p(y2)) + p(y2) (R1 - R2),
//        y1 - y2 = 2 (B - Z0)(q1 - q2) R1 R2,  R1 - R2 = (q2 - q1) R1 R2,
//        q1 - q2 = -sqrt2 t,
//    so  b/b' = sqrt(pi) t R1 R2 [p(y2) - 2 (B - Z0) R1 D],
//    D = (p(y1) - p(y2))/(y1 - y2) <= 0 from a Horner recurrence that runs
//    beside the one for p(y2): both terms are >= 0 and nothing cancels, at
//    any t (this replaces a small-t Taylor branch) and any h (this replaces
//    an asymptotic deep-wing branch).
//  * complement form (q1 < -Z0, i.e. h + t > Z0 sqrt2): b_max - b from the
//    sum above, with erfcx(-q1) = p(y1) R1 from the same recurrences as
//    p(y1) = p(y2) + (y1 - y2) D, then
//    b = b_max - (b_max - b).  Here b >= 0.3 b_max, so the subtraction
//    loses at most two bits, and the upper objective gets b_max - b
//    without cancellation.
//  b and b' themselves leave the normal range deep in the wing (b below
//  2^-1022 keeps fewer significant bits); b/b' and ln b' do not, so ln b is
//  formed as ln b' + ln(b/b') where the logarithmic objective needs it.
struct NBlack {
  double b;      // b(x, s)
  double c;      // b_max - b(x, s)
  double bp;     // db/ds
  double ratio;  // b / b' (difference form; b/b' from b in the complement form)
  double cratio; // (b_max - b) / b' in the complement form, free of the
                 // common factor E (b_max - b and b' underflow together)
  double lnbp;   // ln b' = -(h^2 + t^2)/2 - ln sqrt(2 pi)
  double is;     // 1/s (at the evaluation's precision), for the caller's step
  int form;      // evaluation form taken (kFormDifference or kFormComplement)
};

enum NbForm : int { kFormDifference = 0, kFormComplement = 1 };

// x <= 0, s >= 0, bmax = exp(x/2).  Precision level P: 0 full binary64;
// 1 (the first Householder step) erfcx fit of degree 12, shorter exp,
// one-step reciprocals, ~1e-8 relative in b and in b_max - b; 2 (the
// boundary point of the initial guess) erfcx fit of degree 7 and a
// degree-6 exp, ~1e-5.
// CE (compensated exponent, with P = 0): the exponent -(h^2 + t^2)/2 is
// formed to twice the working precision and its low part carried into E.
// Without it the rounding of h = x/s (a few ulps) is amplified by h^2 in
// E: deep in the wing, where b is tiny, b is then accurate to its inputs'
// conditioning (thousands of ulps at |h| ~ 40) rather than to a few ulps
// of the exact b at the given x and s.  The solvers do not need it: there
// the same error moves the root by only ~1/h^2 of it.
template <int P, bool CE = false>
__host__ __device__ inline NBlack normalised_black_t(double x, double s, double bmax) {
  constexpr bool LO = P >= 1;
  NBlack r;
  if (!(s > 0x1p-1000)) {
    // s = 0, or so small that x/s would overflow: the limit s -> 0, where b
    // vanishes faster than any power of s off the money and b ~ s/sqrt(2 pi)
    // at the money
    const bool atm = x == 0.0;
    r.b = atm ? s * kInvSqrt2Pi : 0.0;
    r.c = bmax - r.b;
    r.bp = atm ? kInvSqrt2Pi : 0.0;
    r.ratio = atm ? s : 0.0;
    r.cratio = __builtin_inf();
    r.lnbp = atm ? -kLnSqrt2Pi : -__builtin_inf();
    r.is = rcp_lo(s);
    r.form = kFormDifference;
    return r;
  }
  r.is = LO ? rcp_lo(s) : rcp(s);
  const double h = x * r.is, t = 0.5 * s;
  double ea = -0.5 * fma(h, h, t * t);
  double E;
  if (CE) {
    // error-free transformations: no product may be contracted into a sum
#pragma clang fp contract(off)
    // x/s = h + hl with hl = (x - h s)/s (the residual is exact in an fma);
    // h^2 = p + pl and t^2 = q + ql exactly; p + q = sm + se by two-sum
    const double hl = fma(-h, s, x) * r.is;
    const double p = h * h, pl = fma(h, h, -p) + 2.0 * h * hl;
    const double q = t * t, ql = fma(t, t, -q);
    const double sm = p + q;
    const double bb = sm - p;
    const double se = (p - (sm - bb)) + (q - bb);
    ea = -0.5 * sm;
    const double ea_lo = -0.5 * (se + (pl + ql));
    const double E0 = fexp(ea);
    E = fma(E0, ea_lo, E0);  // e^{ea + ea_lo} = e^{ea} (1 + ea_lo), |ea_lo| < 2^-52 |ea|
    ea += ea_lo;
  } else {
    E = P == 0 ? fexp(ea) : (P == 1 ? fexp_lo(ea) : fexp_g(ea));
  }
  r.bp = kInvSqrt2Pi * E;
  r.lnbp = ea - kLnSqrt2Pi;
  const double q1 = -(h + t) * kInvSqrt2, q2 = (t - h) * kInvSqrt2;
  const bool comp = q1 < -coef::kErfcxZ0;
  const double z1 = comp ? -q1 : q1;
  constexpr int kDeg = P == 0 ? kErfcxDeg : (P == 1 ? kErfcxLoDeg : kErfcxGDeg);
  constexpr const double* kC = P == 0 ? coef::kErfcx : (P == 1 ? coef::kErfcxLo : coef::kErfcxG);
  constexpr double kB = P == 0 ? coef::kErfcxB : (P == 1 ? coef::kErfcxLoB : coef::kErfcxGB);
  constexpr double kShift = kB - 2.0 * coef::kErfcxZ0;
  // R1 = 1/(z1 + B), R2 = 1/(q2 + B).  At guess precision (P >= 1: the
  // initial guess and the first step, where |h| stays below about 70, so
  // the product below neither overflows nor loses range) both come from
  // one reciprocal of the product; full precision keeps two, which hold for
  // any s above 2^-1000.
  const double a1 = z1 + kB, a2 = q2 + kB;
  double R1, R2;
  if (LO) {
    const double R12 = rcp_lo(a1 * a2);
    R1 = R12 * a2;
    R2 = R12 * a1;
  } else {
    R1 = rcp(a1);
    R2 = rcp(a2);
  }
  const double y1 = (z1 - kShift) * R1, y2 = (q2 - kShift) * R2;
  // B = p(y2), D = (p(y1) - p(y2))/(y1 - y2) by two Horner recurrences
  double B = kC[kDeg], D = 0.0;
#pragma unroll
  for (int i = kDeg - 1; i >= 0; --i) {
    D = fma(D, y1, B);
    B = fma(B, y2, kC[i]);
  }
  if (!comp) {
    constexpr double k2BZ = 2.0 * (kB - coef::kErfcxZ0);
    r.ratio = kSqrtPi * t * R1 * R2 * fma(-k2BZ * R1, D, B);
    r.cratio = __builtin_inf();  // not used in this form
    r.b = r.bp * r.ratio;
    r.c = bmax - r.b;
    r.form = kFormDifference;
  } else {
    // p(y1) = p(y2) + (y1 - y2) D: y1 <= y2 and D <= 0, so both terms are
    // non-negative
    const double A = fma(y1 - y2, D, B);
    const double S = fma(A, R1, B * R2);  // erfcx(-q1) + erfcx(q2)
    r.c = 0.5 * E * S;
    r.cratio = kSqrtPiOver2 * S;
    r.b = bmax - r.c;
    r.ratio = r.b * (LO ? rcp_lo(r.bp) : rcp(r.bp));
    r.form = kFormComplement;
  }
  return r;
}

__host__ __device__ inline NBlack normalised_black(double x, double s, double bmax) {
  return normalised_black_t<0>(x, s, bmax);
}

// b''/b' and b'''/b' as functions of s (closed forms of the derivatives of
// b'(s) = exp(-(x^2/s^2 + s^2/4)/2)/sqrt(2 pi)).
__host__ __device__ inline double nb_d2_over_d1(double x, double s) {
  const double is = rcp(s);
  return x * x * is * is * is - 0.25 * s;
}
__host__ __device__ inline double nb_d3_over_d1(double x, double s, double eta) {
  const double is = rcp(s);
  const double is2 = is * is;
  return eta * eta - 3.0 * x * x * is2 * is2 - 0.25;
}

}  // namespace fv
