// fv_quote.h -- per-quote pre-processing, post-processing, Greeks and the
// implied-volatility adjoint, shared by every kernel.
//
// Pre-processing (the paper's section 4: flags normalised, inputs validated;
// section 2.4: a Black-76 price is the discounted mid and the same r both
// discounts and inverts):
//   F  = forward:  Black-76 input, S e^{rT} (Black-Scholes),
//                  S e^{(r-q)T} (Black-Scholes-Merton);   D = e^{-rT};
//   Pu = price / D  (undiscounted),
//   I  = max(theta (F - K), 0),  M = F (call) or K (put);
//   Pu <  I  -> BELOW_INTRINSIC,  Pu == I -> AT_INTRINSIC (sigma = 0),
//   Pu >= M  -> ABOVE_MAX;  non-finite or non-positive F/S, K, T -> INVALID.
// Solvable quotes are reduced to an out-of-the-money call by put-call
// parity (Pu -= I, theta -> -theta when in the money) and normalised:
//   x = theta ln(F/K) <= 0,  beta = Pu / sqrt(F K),  s = sigma sqrt(T).
#pragma once

#include "fv_lbr.h"

namespace fv {

enum Model : int { kBlack76 = 0, kBlackScholes = 1, kBlackScholesMerton = 2 };
enum QuoteStatus : uint8_t {
  kQOk = 0,
  kQAtIntrinsic = 1,
  kQBelowIntrinsic = 2,
  kQAboveMax = 3,
  kQInvalid = 4,
  kQNotConverged = 5,
};

struct Reduced {
  double F, D;
  double isqrtT;   // 1/sqrt(T): sigma = s isqrtT
  double x, beta;  // normalised out-of-the-money call: x <= 0, 0 < beta < e^{x/2}
  double bmax;     // e^{x/2} = min(F, K)/sqrt(F K)
  double lnb;      // ln beta, to full relative precision also where beta is below
                   // the normal range (or underflowed) for an out-of-the-money quote
  uint8_t status;
};

// Finite test by classification (v_cmp_class), never by arithmetic: with
// contraction on, v - v == 0 for a product v = a b compiles to
// fma(a, b, -v) == 0, the product's rounding error, which is rarely 0.
__host__ __device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

// sqrt(T) for finite T > 0 as T / sqrt(T) from the refined reciprocal
// square root, with T scaled by 2^200 first when it is so small that
// v_rsq_f64 could see a denormal
__host__ __device__ inline double sqrt_pos(double T) {
  const bool tiny = T < 1e-290;
  const double Ts = tiny ? T * 0x1p+200 : T;
  return Ts * rsqrt(Ts) * (tiny ? 0x1p-100 : 1.0);
}

// 1/sqrt(T) for finite T > 0, with the same scaling of tiny T
__host__ __device__ inline double rsqrt_pos(double T) {
  const bool tiny = T < 1e-290;
  const double Ts = tiny ? T * 0x1p+200 : T;
  return rsqrt(Ts) * (tiny ? 0x1p+100 : 1.0);
}

// e^{a b} with the rounding error of the exponent carried into the result:
// a b = p + e exactly (p = fl(a b), e = fma(a, b, -p)) and e^{p + e} =
// e^p (1 + e) to first order (|e| <= 2^-53 |p|).  Over long maturities r T
// reaches tens, where dropping e would put tens of ulps into the forward or
// the discount factor, errors that the inputs' own conditioning does not
// cover (the exact sensitivity to r cancels between forward and discount).
__host__ __device__ inline double fexp_prod(double a, double b) {
  const double p = a * b;
  const double e = fma(a, b, -p);
  const double E = fexp(p);
  return fma(E, e, E);
}

// e^{(r - q) T}, carrying the rounding of r - q as well (Knuth's two-sum:
// r - q = c + ce exactly)
__host__ __device__ inline double fexp_carry(double r, double q, double T) {
  const double c = r - q;
  const double bb = c - r;
  const double ce = (r - (c - bb)) + (-q - bb);
  const double p = c * T;
  const double e = fma(c, T, -p) + ce * T;
  const double E = fexp(p);
  return fma(E, e, E);
}

__host__ __device__ inline double forward_of(int model, double fs, double T, double r,
                                             double q) {
  if (model == kBlack76) return fs;
  return fs * (model == kBlackScholesMerton ? fexp_carry(r, q, T) : fexp_prod(r, T));
}

// ln(F/K) from the ratio while F/K is a normal number, else from the two
// logarithms (|ln(F/K)| beyond about 708, or an operand the refined
// reciprocal cannot take: the comparisons fail on a NaN ratio).
__host__ __device__ inline double log_moneyness(double F, double K) {
  const double fk = F * rcp(K);
  return (fk > kDblMin && fk < 0x1p1023) ? flog(fk) : flog(F) - flog(K);
}

__host__ __device__ inline Reduced reduce_quote(int model, double price, double fs, double K,
                                                double T, double r, double q, int theta) {
  // One exit: every lane computes every field and the status is decided at
  // the end, in the order of the checks below (invalid input first).  The
  // fields of a quote whose status is not OK are meaningless and no caller
  // reads them; early returns would instead make every path set defaults.
  Reduced o;
  // S/F and K must be normal numbers (the refined hardware reciprocals
  // below need normal operands); so must the forward
  const bool ok_in = finite_d(price) && finite_d(fs) && finite_d(K) && finite_d(T) &&
                     finite_d(r) && finite_d(q) && fs >= kDblMin && K >= kDblMin && T > 0.0 &&
                     (theta == 1 || theta == -1);
  const double F = forward_of(model, fs, T, r, q);
  const bool ok_f = F >= kDblMin && finite_d(F);
  const double D = fexp_prod(-r, T);
  const double Pu = price * fexp_prod(r, T);
  const double dth = (double)theta;
  const double I = fmax(dth * (F - K), 0.0);  // intrinsic value (the sign flip is exact)
  const double M = theta > 0 ? F : K;
  o.F = F;
  o.D = D;
  o.isqrtT = rsqrt_pos(T);
  // in the money: parity to out of the money
  const double th = I > 0.0 ? -dth : dth;
  o.x = th * log_moneyness(F, K);
  // 1/sqrt(F K) as two factors: F K itself leaves the binary64 range once F
  // and K are beyond about 1e+-154, while the normalised quantities do not
  // (and scaling price, F and K by an even power of two scales both factors
  // exactly, so the result is bitwise homogeneous of degree 0)
  const double isq = rsqrt(F) * rsqrt(K);
  o.beta = (Pu - I) * isq;
  o.bmax = fmin(F, K) * isq;
  if (o.beta < 0x1p-1000 && I == 0.0) {
    // out of the money with a price too small for beta to keep full precision
    // in binary64: ln beta = ln P + r T - ln(F K)/2 from the price itself
    o.lnb = flog(price) + r * T - 0.5 * (flog(F) + flog(K));
  } else {
    o.lnb = flog(o.beta);
  }
  // the normalised price can round onto its bound even when Pu < M
  uint8_t st = o.beta < o.bmax ? kQOk : kQAboveMax;
  if (Pu >= M) st = kQAboveMax;
  if (Pu == I) st = kQAtIntrinsic;
  if (Pu < I) st = kQBelowIntrinsic;
  if (!(ok_in && ok_f)) st = kQInvalid;
  o.status = st;
  return o;
}

// Accurate Phi(a) for either sign of a.
__host__ __device__ inline double norm_cdf_signed(double a) { return norm_cdf(a); }

// Raw per-unit Greeks at sigma (paper section 3: get_all_greeks returns all
// five from one d1/d2 evaluation):
//   delta = dP/dS (dP/dF for Black-76), gamma = d2P/dS2, vega = dP/dsigma,
//   theta = -dP/dT per year, rho = dP/dr (Black-76: at fixed F).
// `price` is the option price at sigma (input or recomputed by the caller).
struct Greeks {
  double delta, gamma, vega, theta, rho;
};

// Terms every closed form below shares, computed once: s = sigma sqrt(T),
// d1 = ln(F/K)/s + s/2, d2 = d1 - s, Phi(theta d1), Phi(theta d2), phi(d1)
// and the discounted forward D F (= S e^{-qT} for Black-Scholes(-Merton)).
struct BsTerms {
  double sqT, s, d1, d2, N1, N2, n1, DF;
};

__host__ __device__ inline BsTerms bs_terms(double F, double K, double D, double sigma, double T,
                                            int theta) {
  BsTerms c;
  c.sqT = sqrt_pos(T);
  c.s = sigma * c.sqT;
  c.d1 = log_moneyness(F, K) / c.s + 0.5 * c.s;
  c.d2 = c.d1 - c.s;
  c.N1 = norm_cdf(theta * c.d1);
  c.N2 = norm_cdf(theta * c.d2);
  c.n1 = norm_pdf(c.d1);
  c.DF = D * F;
  return c;
}

__host__ __device__ inline Greeks greeks_from(const BsTerms& c, int model, double fs, double K,
                                              double T, double r, double q, double sigma,
                                              int theta, double F, double D, double price) {
  Greeks g;
  g.vega = c.DF * c.n1 * c.sqT;
  const double decay = 0.5 * sigma * c.DF * c.n1 / c.sqT;  // -dP/dT from the time value
  if (model == kBlack76) {
    g.delta = theta * D * c.N1;
    g.gamma = D * c.n1 / (F * c.s);
    g.theta = r * price - decay;
    g.rho = -T * price;
  } else {
    const double qy = (model == kBlackScholesMerton) ? q : 0.0;
    const double Dq = c.DF / fs;  // e^{-qT}
    g.delta = theta * Dq * c.N1;
    g.gamma = Dq * c.n1 / (fs * c.s);
    g.theta = -decay - theta * r * K * D * c.N2 + theta * qy * c.DF * c.N1;
    g.rho = theta * K * T * D * c.N2;
  }
  return g;
}

__host__ __device__ inline Greeks greeks_at(int model, double fs, double K, double T, double r,
                                            double q, double sigma, int theta, double F,
                                            double D, double price) {
  return greeks_from(bs_terms(F, K, D, sigma, T, theta), model, fs, K, T, r, q, sigma, theta, F,
                     D, price);
}

// Partial derivatives of the price at fixed sigma:
//   d/dfs = delta, d/dK = -theta D Phi(theta d2), d/dT = -(Greek theta),
//   d/dr = rho, d/dq = -theta T D F Phi(theta d1) (Black-Scholes-Merton
//   only), d/dsigma = vega.
struct PricePartials {
  double dfs, dK, dT, dr, dq, dsigma;
};

__host__ __device__ inline PricePartials price_partials(int model, double fs, double K,
                                                        double T, double r, double q,
                                                        double sigma, int theta, double F,
                                                        double D, double price) {
  PricePartials o;
  const BsTerms c = bs_terms(F, K, D, sigma, T, theta);
  const Greeks g = greeks_from(c, model, fs, K, T, r, q, sigma, theta, F, D, price);
  o.dfs = g.delta;
  o.dK = -theta * D * c.N2;
  o.dT = -g.theta;
  o.dr = g.rho;
  o.dq = (model == kBlackScholesMerton) ? -theta * T * c.DF * c.N1 : 0.0;
  o.dsigma = g.vega;
  return o;
}

// Implicit-function adjoint of the implied volatility (the paper's section 3,
// "Differentiable IV"): with vega = dP/dsigma,
//   dsigma/dP = 1/vega,   dsigma/dX = -(dP/dX at fixed sigma)/vega,
// X in (S or F, K, T, r, q).  Returns the six partials.
struct IvGrad {
  double dP, dfs, dK, dT, dr, dq;
};

__host__ __device__ inline IvGrad iv_gradient(int model, double fs, double K, double T,
                                              double r, double q, double sigma, int theta,
                                              double price) {
  IvGrad o;
  const double F = forward_of(model, fs, T, r, q);
  const double D = fexp_prod(-r, T);
  const PricePartials pp = price_partials(model, fs, K, T, r, q, sigma, theta, F, D, price);
  const double iv = 1.0 / pp.dsigma;
  o.dP = iv;
  o.dfs = -pp.dfs * iv;
  o.dK = -pp.dK * iv;
  o.dT = -pp.dT * iv;
  o.dr = -pp.dr * iv;
  o.dq = -pp.dq * iv;
  return o;
}

// Price at sigma from the normalised Black function (accurate in the wings):
// price = D sqrt(F K) b(x, s, theta), with b of a put or an in-the-money
// option obtained from the out-of-the-money call by parity.
__host__ __device__ inline double price_at(double F, double K, double D, double sigma,
                                           double sqrtT, int theta) {
  const double lx = log_moneyness(F, K);
  // out-of-the-money side: x_otm <= 0
  const bool itm = theta * lx > 0.0;
  const double x = -fabs(lx);
  const double bmax = fexp(0.5 * x);
  const NBlack nb = normalised_black(x, sigma * sqrtT, bmax);
  const double sq = sqrt(F) * sqrt(K);  // F K may leave the binary64 range
  double p = D * sq * nb.b;
  if (itm) p += D * (theta > 0 ? (F - K) : (K - F));
  return p;
}

}  // namespace fv
