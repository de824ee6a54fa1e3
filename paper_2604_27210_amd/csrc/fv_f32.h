// fv_f32.h -- binary32 normalised Black evaluator, reduction and Halley
// solver: the paper's Halley path for label pipelines that train in float32
// and need fewer digits than the reference path (section 2.2, "Dual-Solver
// Design").  Same method as the binary64 Halley path (fv_lbr.h), in float:
//   * b(x, s) from one polynomial erfcx fit in a Moebius variable, the
//     difference erfcx(q1) - erfcx(q2) taken as a divided difference (no
//     cancellation at small t or deep in the wing), the complement
//     b_max - b for h + t > 1/sqrt2;
//   * exp and log from a two-part ln 2 reduction with the hardware 2^x and
//     an atanh series, reciprocals and square roots from the hardware
//     single-precision instructions (about 1 ulp each);
//   * Brenner-Subrahmanyam start, at most 8 Halley steps with the far-field
//     log-Newton step and the sign bracket, bisection for the lanes that fail
//     the convergence check.
// Domain: a normalised price beta below 2^-100 is left to the binary64 path
// (the caller gets NaN and FV_Q_NOT_CONVERGED): binary32 keeps full relative
// precision only down to 2^-126, and the evaluator's intermediate products
// need the margin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_coeffs.h"

namespace fv32 {

constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;
constexpr float kSqrt2Pi = 2.50662827463100050f;
constexpr float kSqrtPi = 1.77245385090551603f;
constexpr float kLog2E = 1.44269504088896341f;
constexpr float kLn2Hi = 0.693145751953125f;      // 15 significant bits: n kLn2Hi exact
constexpr float kLn2Lo = 1.42860682030941723e-6f;  // ln 2 - kLn2Hi
constexpr float kBetaMin = 7.8886090522101181e-31f;  // 2^-100
constexpr float kFltMin = 1.17549435082228751e-38f;  // smallest normal binary32

// by classification, not v - v == 0 (contraction would turn that into the
// rounding error of a product)
__host__ __device__ inline bool finite(float v) { return __builtin_isfinite(v); }

__host__ __device__ inline float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

__host__ __device__ inline float rsqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// e^x: x = n ln2 + r, |r| <= ln2/2 (ln 2 in two parts), e^r = 2^(r log2 e)
// from the hardware power of two; arguments below -104 give 0.
__host__ __device__ inline float fexp(float x) {
  x = fmaxf(x, -104.0f);
  const float n = rintf(x * kLog2E);
  const float r = fmaf(-n, kLn2Lo, fmaf(-n, kLn2Hi, x));
#if defined(__HIP_DEVICE_COMPILE__)
  const float er = __builtin_amdgcn_exp2f(r * kLog2E);
#else
  const float er = exp2f(r * kLog2E);
#endif
  return ldexpf(er, (int)n);
}

// ln x for positive finite x: x = 2^e m, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 0.1716: four series terms
// reach binary32 precision, with full relative precision near x = 1.
__host__ __device__ inline float flog(float x) {
  int e;
  float m = frexpf(x, &e);
  if (m < 0.70710678f) {
    m += m;
    --e;
  }
  const float f = (m - 1.0f) * rcp(m + 1.0f);
  const float z = f * f;
  float S = 1.0f / 9.0f;
  S = fmaf(S, z, 1.0f / 7.0f);
  S = fmaf(S, z, 1.0f / 5.0f);
  S = fmaf(S, z, 1.0f / 3.0f);
  const float f2 = f + f;
  const float de = (float)e;
  return fmaf(de, kLn2Hi, fmaf(de, kLn2Lo, fmaf(f2 * z, S, f2)));
}

constexpr int kDeg = (int)(sizeof(fv::coef::kErfcxF32) / sizeof(double)) - 1;

struct NBlack {
  float b, c, bp;
};

// b(x, s), b_max - b and b' for x <= 0 (see the binary64 evaluator).
__host__ __device__ inline NBlack normalised_black(float x, float s, float bmax) {
  NBlack r;
  if (!(s > 1e-30f)) {
    const bool atm = x == 0.0f;
    r.b = atm ? s * kInvSqrt2Pi : 0.0f;
    r.c = bmax - r.b;
    r.bp = atm ? kInvSqrt2Pi : 0.0f;
    return r;
  }
  const float h = x * rcp(s), t = 0.5f * s;
  const float E = fexp(-0.5f * fmaf(h, h, t * t));
  r.bp = kInvSqrt2Pi * E;
  const float q1 = -(h + t) * kInvSqrt2, q2 = (t - h) * kInvSqrt2;
  constexpr float kZ0 = (float)fv::coef::kErfcxZ0;
  constexpr float kB = (float)fv::coef::kErfcxF32B;
  constexpr float kShift = kB - 2.0f * kZ0;
  const bool comp = q1 < -kZ0;
  const float z1 = comp ? -q1 : q1;
  const float R1 = rcp(z1 + kB), R2 = rcp(q2 + kB);
  const float y1 = (z1 - kShift) * R1, y2 = (q2 - kShift) * R2;
  float B = (float)fv::coef::kErfcxF32[kDeg], D = 0.0f;
#pragma unroll
  for (int i = kDeg - 1; i >= 0; --i) {
    D = fmaf(D, y1, B);
    B = fmaf(B, y2, (float)fv::coef::kErfcxF32[i]);
  }
  if (!comp) {
    constexpr float k2BZ = 2.0f * (kB - kZ0);
    r.b = r.bp * (kSqrtPi * t * R1 * R2 * fmaf(-k2BZ * R1, D, B));
    r.c = bmax - r.b;
  } else {
    const float A = fmaf(y1 - y2, D, B);  // p(y1); both terms >= 0
    r.c = 0.5f * E * fmaf(A, R1, B * R2);
    r.b = bmax - r.c;
  }
  return r;
}

// Model reduction (as fv::reduce_quote, in binary32).  Status codes are the
// library's FV_Q_* values.
struct Reduced {
  float x, beta, bmax, lnb, sqrtT;
  uint8_t status;
};

// e^{a b} and e^{(r - q) T} with the rounding of the exponent carried into
// the result, as in the binary64 path: a b = p + e exactly, e^{p + e} =
// e^p (1 + e) to first order (and r - q = c + ce exactly by two-sum).
__host__ __device__ inline float fexp_prod(float a, float b) {
  const float p = a * b;
  const float e = fmaf(a, b, -p);
  const float E = fexp(p);
  return fmaf(E, e, E);
}
__host__ __device__ inline float fexp_carry(float r, float q, float T) {
  const float c = r - q;
  const float bb = c - r;
  const float ce = (r - (c - bb)) + (-q - bb);
  const float p = c * T;
  const float e = fmaf(c, T, -p) + ce * T;
  const float E = fexp(p);
  return fmaf(E, e, E);
}

__host__ __device__ inline Reduced reduce_quote(int model, float price, float fs, float K,
                                                float T, float r, float q, int theta) {
  Reduced o;
  o.x = o.beta = o.bmax = o.lnb = o.sqrtT = 0.0f;
  const bool ok_in = finite(price) && finite(fs) && finite(K) && finite(T) && finite(r) &&
                     finite(q) && fs >= kFltMin && K >= kFltMin && T > 0.0f &&
                     (theta == 1 || theta == -1);
  if (!ok_in) { o.status = 4; return o; }
  const float F = model == 0 ? fs : fs * (model == 2 ? fexp_carry(r, q, T) : fexp_prod(r, T));
  if (!(F >= kFltMin && finite(F))) { o.status = 4; return o; }
  const float Pu = price * fexp_prod(r, T);
  const float I = theta > 0 ? fmaxf(F - K, 0.0f) : fmaxf(K - F, 0.0f);
  const float M = theta > 0 ? F : K;
  o.sqrtT = sqrtf(T);
  if (Pu < I) { o.status = 2; return o; }
  if (Pu == I) { o.status = 1; return o; }
  if (Pu >= M) { o.status = 3; return o; }
  const int th = (I > 0.0f) ? -theta : theta;
  // ln(F/K) from the ratio, or from the two logarithms where F/K leaves the
  // binary32 normal range (|ln(F/K)| beyond about 87)
  const float fk = F * rcp(K);
  float lx;
  if (fk > kFltMin && fk < 0x1p127f)
    lx = flog(fk);
  else
    lx = flog(F) - flog(K);
  o.x = th > 0 ? lx : -lx;
  const float isq = rsqrt(F) * rsqrt(K);  // F K leaves binary32 beyond about 1e+-19
  o.beta = (Pu - I) * isq;
  o.bmax = fminf(F, K) * isq;
  o.status = (o.beta < o.bmax) ? 0 : 3;
  if (o.status == 0 && !(o.beta >= kBetaMin)) o.status = 5;  // outside the binary32 domain
  o.lnb = o.status == 0 ? flog(o.beta) : 0.0f;
  return o;
}

struct HalleyState {
  float s, lo, hi;
  bool converged;
};

// Halley on b(s) - beta from s0 = sqrt(2 pi) beta, as fv::halley_solve:
// far-field log-Newton step in u = 1/s^2 when the residual is negative and
// the Halley factor below 1/2, a sign bracket, a lane stops once its step
// is below 2^-22 s.  Converged: last |step| <= 1e-5 s and
// |b - beta| <= 1e-5 beta.
__host__ __device__ __attribute__((always_inline)) inline HalleyState halley_solve(
    float x, float beta, float bmax, float ln_beta, int steps) {
  HalleyState st;
  st.lo = 0.0f;
  st.hi = 3.0e38f;
  float s = kSqrt2Pi * beta;
  float ds = 0.0f, res = 0.0f;
  for (int k = 0; k < steps; ++k) {
    const NBlack nb = normalised_black(x, s, bmax);
    res = nb.b - beta;
    if (res < 0.0f) st.lo = s; else st.hi = s;
    const float nu = -res * rcp(nb.bp);
    const float is = rcp(s);
    const float eta = x * x * is * is * is - 0.25f * s;
    const float hf = rcp(1.0f + 0.5f * eta * nu);
    float sn = s + nu * hf;
    if (res < 0.0f && !(hf >= 0.5f) && x < 0.0f) {
      float un = -1.0f;
      if (nb.b > 1e-36f) {
        const float dLdu = -0.5f * nb.bp * rcp(nb.b) * s * s * s;
        un = fmaf((ln_beta - flog(nb.b)) * rcp(dLdu), 1.0f, is * is);
      }
      sn = (un > 0.0f && un < 1e38f) ? rsqrt(un) : fmaxf(2.0f * s, -x * rsqrt(-2.0f * ln_beta));
    }
    if (!(sn >= st.lo && sn <= st.hi)) {
      if (st.hi >= 3.0e38f) sn = 2.0f * s + 1e-3f;
      else if (st.lo > 0.0f) sn = sqrtf(st.lo) * sqrtf(st.hi);
      else sn = 0.5f * st.hi;
    }
    ds = sn - s;
    s = sn;
    if (fabsf(ds) <= 2.384185791e-7f * s) break;
  }
  st.s = s;
  st.converged = fabsf(ds) <= 1e-5f * s && fabsf(res) <= 1e-5f * beta;
  return st;
}

// Geometric bisection on s inside [lo, hi] to rel_tol (midpoints as
// sqrt(lo) sqrt(hi)).
__host__ __device__ inline float bisection_solve(float x, float beta, float bmax, float lo,
                                                 float hi, float rel_tol) {
  // an end the caller's bracket did not fix: far below any root, and far
  // above it (b_max - b(s) is below b_max 2^-24 once s exceeds ~12 + |x|/10)
  if (!(lo > 0.0f)) lo = 1e-30f;
  if (!(hi < 3.0e38f)) hi = 1e3f;
  for (int k = 0; k < 100 && hi - lo > rel_tol * hi; ++k) {
    const float mid = sqrtf(lo) * sqrtf(hi);
    const NBlack nb = normalised_black(x, mid, bmax);
    if (nb.b < beta) lo = mid; else hi = mid;
  }
  return sqrtf(lo) * sqrtf(hi);
}

}  // namespace fv32
