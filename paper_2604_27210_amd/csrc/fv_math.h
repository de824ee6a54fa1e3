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
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kEps = 2.220446049250313e-16;

// Branch thresholds of the normalised Black evaluator.
//   small-t Taylor branch:      t < kTauSmall  (= 2 eps^{1/16})
//   asymptotic (deep wing):     h < kHLarge and h + t < kHLarge + kTauSmall
constexpr double kTauSmall = 0.21022410381342863;
constexpr double kHLarge = -10.0;

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
  const double f = (m - 1.0) / (m + 1.0);
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

// ----------------------------------------------------------------- erfcx
// erfcx(z) = exp(z^2) erfc(z) for z >= 0, one branch-free polynomial in
// y = (z - K)/(z + K) (fitted coefficients, fv_coeffs.h).
__host__ __device__ inline double erfcx_nonneg(double z) {
  const double R = rcp(z + coef::kErfcxK);
  const double y = (z - coef::kErfcxK) * R;
  double p = coef::kErfcx[23];
#pragma unroll
  for (int i = 22; i >= 0; --i) p = fma(p, y, coef::kErfcx[i]);
  return p * R;
}

// Standard normal density and CDF.  Phi goes through erfcx so that the lower
// tail keeps full relative precision (paper section 2.3 evaluates the CDF
// through the complementary error function for the same reason).
__host__ __device__ inline double norm_pdf(double z) { return kInvSqrt2Pi * fexp(-0.5 * z * z); }

__host__ __device__ inline double norm_cdf(double z) {
  const double a = fabs(z) * kInvSqrt2;
  const double tail = 0.5 * fexp(-0.5 * z * z) * erfcx_nonneg(a);  // Phi(-|z|)
  return z < 0.0 ? tail : 1.0 - tail;
}

// Inverse standard normal CDF for p in (0, 1/2] (returns a value <= 0).
// Accurate to ~1e-13 relative; only initial guesses use it.
__host__ __device__ inline double inv_norm_cdf_lower(double p) {
  double z;
  if (p >= coef::kPhiInvSplit) {
    const double q = p - 0.5, w = q * q;
    double num = coef::kPhiInvCentralP[6], den = coef::kPhiInvCentralQ[6];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      num = fma(num, w, coef::kPhiInvCentralP[i]);
      den = fma(den, w, coef::kPhiInvCentralQ[i]);
    }
    z = q * fdiv(num, den);
  } else {
    const double r = sqrt(-2.0 * flog(p));
    double num = coef::kPhiInvTailP[7], den = coef::kPhiInvTailQ[7];
#pragma unroll
    for (int i = 6; i >= 0; --i) {
      num = fma(num, r, coef::kPhiInvTailP[i]);
      den = fma(den, r, coef::kPhiInvTailQ[i]);
    }
    z = fdiv(num, den);
  }
  return z;
}

// ---------------------------------------------------- normalised Black
// b(x,s)/b'(x,s) = Y(h+t) - Y(h-t) with Y(z) = Phi(z)/phi(z), and
// b'(x,s) = db/ds = exp(-(h^2+t^2)/2)/sqrt(2 pi).  Three evaluation forms:
//
//  * erfcx form: with q1 = -(h+t)/sqrt2, q2 = (t-h)/sqrt2 >= 0 and
//    E = exp(-(h^2+t^2)/2),
//        b       = E/2 [erfcx(q1) - erfcx(q2)]     when q1 >= 0,
//        b_max-b = E/2 [erfcx(-q1) + erfcx(q2)]    when q1 <  0,
//    so every erfcx argument is >= 0 and the complement b_max - b, which the
//    upper objective needs, never suffers cancellation.
//  * small-t form: the odd Taylor series in t of Y(h+t) - Y(h-t),
//        2 sum_{k odd} t^k Y^{(k)}(h)/k!,
//    with Y^{(k)} from Y' = 1 + hY, Y^{(k+1)} = h Y^{(k)} + k Y^{(k-1)}; it
//    removes the cancellation of the erfcx difference when t is small.
//  * asymptotic form (h << 0): with A = -(h+t), B = t-h, rho = A/B, the
//    asymptotic series Y(z) ~ sum_n (-1)^n (2n-1)!! |z|^{-(2n+1)} gives
//        Y(h+t) - Y(h-t) = 2t/(A B) sum_n (-1)^n (2n-1)!! A^{-2n} G_n(rho),
//        G_n = 1 + rho + ... + rho^{2n},
//    a sum of positive G_n with an alternating, decreasing asymptotic
//    factor: no cancellation between A- and B-terms.
struct NBlack {
  double b;   // b(x, s)
  double c;   // b_max - b(x, s)
  double bp;  // db/ds
  int form;   // evaluation form taken (kFormAsymptotic ... kFormComplement)
};

enum NbForm : int { kFormAsymptotic = 0, kFormSmallT = 1, kFormErfcx = 2, kFormComplement = 3 };

// y0 = Y(h) = sqrt(pi/2) erfcx(-h/sqrt2) for h <= 0.
__host__ __device__ inline double nb_small_t_ratio(double h, double t, double y0) {
  double ym = y0;                 // Y^{(k-1)}
  double yk = fma(h, y0, 1.0);    // Y^{(1)}
  const double t2 = t * t;
  // sum_{j>=0} t^{2j} Y^{(2j+1)} / (2j+1)!
  double sum = yk;
  double tp = 1.0;                // t^{2j} / (2j+1)!
#pragma unroll
  for (int k = 1; k < 17; k += 2) {
    // advance two orders: Y^{(k+1)}, Y^{(k+2)}
    const double y1 = fma(h, yk, k * ym);
    const double y2 = fma(h, y1, (k + 1) * yk);
    ym = y1;
    yk = y2;
    tp *= t2 * (1.0 / ((k + 1) * (k + 2)));
    sum = fma(tp, yk, sum);
  }
  return 2.0 * t * sum;
}

__host__ __device__ inline double nb_asymptotic_ratio(double h, double t) {
  const double A = -(h + t), B = t - h;
  const double iB = rcp(B), iA = rcp(A);
  const double rho = A * iB, a = iA * iA;  // 1/A^2 may underflow to 0, never inf
  double coefn = 1.0, G = 1.0, rp = rho, sum = 1.0;
  const double onep = 1.0 + rho, rho2 = rho * rho;
#pragma unroll
  for (int n = 1; n <= 24; ++n) {
    coefn *= -(2 * n - 1) * a;
    G = fma(rp, onep, G);
    rp *= rho2;
    sum = fma(coefn, G, sum);
  }
  return 2.0 * t * iA * iB * sum;
}

// x <= 0, s >= 0, bmax = exp(x/2).  The small-t and erfcx forms share their
// first erfcx call (argument -h/sqrt2 or |q1|), so a wave mixing the two
// forms evaluates two erfcx, not three.
__host__ __device__ inline NBlack normalised_black(double x, double s, double bmax) {
  NBlack r;
  r.form = kFormErfcx;
  if (!(s > 0.0)) {
    r.b = 0.0;
    r.c = bmax;
    r.bp = (x == 0.0) ? kInvSqrt2Pi : 0.0;
    return r;
  }
  const double h = x * rcp(s), t = 0.5 * s;
  const double E = fexp(-0.5 * fma(h, h, t * t));
  r.bp = kInvSqrt2Pi * E;
  const bool asym = h < kHLarge && h + t < kHLarge + kTauSmall;
  if (asym) {
    r.b = r.bp * nb_asymptotic_ratio(h, t);
    r.c = bmax - r.b;
    r.form = kFormAsymptotic;
    return r;
  }
  const bool small = t < kTauSmall;
  const double q1 = -(h + t) * kInvSqrt2;
  const double e1 = erfcx_nonneg(small ? -h * kInvSqrt2 : fabs(q1));
  if (small) {
    r.b = r.bp * nb_small_t_ratio(h, t, kSqrtPiOver2 * e1);
    r.c = bmax - r.b;
    r.form = kFormSmallT;
  } else {
    const double e2 = erfcx_nonneg((t - h) * kInvSqrt2);
    if (q1 >= 0.0) {
      r.b = 0.5 * E * (e1 - e2);
      r.c = bmax - r.b;
    } else {
      r.c = 0.5 * E * (e1 + e2);
      r.b = bmax - r.c;
      r.form = kFormComplement;
    }
  }
  return r;
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
