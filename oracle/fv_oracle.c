/*
 * fv_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU oracle for European-option pricing, Greeks,
 * implied volatility and the implied-volatility gradient under Black-76,
 * Black-Scholes and Black-Scholes-Merton (the three models of the paper's
 * section 3, "Capabilities").  It exists so the test-suite, the smoke check
 * and the CPU-baseline timing can check the GPU library against definitions
 * a reader can verify by eye.  The product path never links, loads or calls
 * it, and it shares no code, header, table or constant with that path.
 *
 * Arithmetic: every model quantity is evaluated in IEEE binary128
 * (__float128, libquadmath) and rounded to double only at the end.  The
 * implied volatility is, by the paper's section 1, the unique sigma at which
 * the model price equals the observed price; the oracle computes exactly
 * that root of the textbook price formula, to ~1e-30 relative, with a
 * safeguarded Newton/bisection iteration.  It deliberately does NOT follow
 * the fast "Let's Be Rational" steps of the paper's section 2.2: that method
 * converges to the same root, so the root itself is the reference.
 *
 * The per-quote status (at intrinsic, below intrinsic, above the maximum,
 * invalid) is an integer decided by floating point, so it is decided here in
 * binary64, with the same comparisons the GPU library documents:
 *   F = forward (Black-76 input; S*exp((r-q)T) otherwise), D = exp(-rT),
 *   Pu = price/D, I = max(theta*(F-K), 0), M = F (call) or K (put);
 *   Pu < I -> below, Pu == I -> at intrinsic, Pu >= M -> above maximum.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC fv_oracle.c
 *        -lquadmath -lm
 */
#include <float.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 qr;

/* model numbering used by this file's entry points */
enum { ORC_B76 = 0, ORC_BS = 1, ORC_BSM = 2 };
/* per-quote status numbering used by this file's entry points */
enum {
    ORC_OK = 0,
    ORC_AT_INTRINSIC = 1,
    ORC_BELOW_INTRINSIC = 2,
    ORC_ABOVE_MAX = 3,
    ORC_INVALID = 4,
    /* binary64 comparisons say "solvable" but in exact arithmetic the price
     * sits on or outside the no-arbitrage bounds, so no finite positive root
     * exists: a boundary-ambiguous quote */
    ORC_NO_EXACT_ROOT = 8,
    /* the root iteration hit its cap (a defect of this file if it occurs) */
    ORC_ROOT_CAP = 9
};

static const qr Q_SQRT2 = 1.41421356237309504880168872420969807856967Q;
static const qr Q_SQRT2PI = 2.50662827463100050241576528481104525300698Q;

/* Standard normal CDF through the complementary error function, which keeps
 * full relative precision in the lower tail (paper section 2.3). */
static qr q_Phi(qr z) { return 0.5Q * erfcq(-z / Q_SQRT2); }
static qr q_phi(qr z) { return expq(-0.5Q * z * z) / Q_SQRT2PI; }

/* ------------------------------------------------------------------------ */
/* Model inputs                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int model;          /* ORC_B76 / ORC_BS / ORC_BSM */
    qr fs, K, T, r, q;  /* F for Black-76, spot S otherwise */
    int theta;          /* +1 call, -1 put */
} qin;

static qr q_forward(const qin *a)
{
    if (a->model == ORC_B76) return a->fs;
    qr carry = (a->model == ORC_BSM) ? (a->r - a->q) : a->r;
    return a->fs * expq(carry * a->T);
}
static qr q_discount(const qin *a) { return expq(-a->r * a->T); }
static qr q_divyield(const qin *a) { return a->model == ORC_BSM ? a->q : 0.0Q; }

/* ------------------------------------------------------------------------ */
/* Textbook prices (paper section 3: fast_black, fast_black_scholes,         */
/* fast_black_scholes_merton; Black-76 price is the discounted one,          */
/* section 2.4).                                                             */
/* ------------------------------------------------------------------------ */
static qr q_price(const qin *a, qr sigma)
{
    const int th = a->theta;
    qr D = q_discount(a);
    if (sigma <= 0) {
        qr F = q_forward(a);
        qr iv = th * (F - a->K);
        return D * (iv > 0 ? iv : 0);
    }
    qr sd = sigma * sqrtq(a->T);
    if (a->model == ORC_B76) {
        /* e^{-rT} theta [F Phi(theta d1) - K Phi(theta d2)] */
        qr d1 = (logq(a->fs / a->K) + 0.5Q * sigma * sigma * a->T) / sd;
        qr d2 = d1 - sd;
        return D * th * (a->fs * q_Phi(th * d1) - a->K * q_Phi(th * d2));
    }
    /* theta [S e^{-qT} Phi(theta d1) - K e^{-rT} Phi(theta d2)] */
    qr qy = q_divyield(a);
    qr d1 = (logq(a->fs / a->K) + (a->r - qy + 0.5Q * sigma * sigma) * a->T) / sd;
    qr d2 = d1 - sd;
    return th * (a->fs * expq(-qy * a->T) * q_Phi(th * d1) - a->K * D * q_Phi(th * d2));
}

/* d1, d2 of the textbook formula (both models share the forward form). */
static void q_d12(const qin *a, qr sigma, qr *d1, qr *d2)
{
    qr F = q_forward(a);
    qr sd = sigma * sqrtq(a->T);
    *d1 = (logq(F / a->K) + 0.5Q * sd * sd) / sd;
    *d2 = *d1 - sd;
}

/* Greeks as raw per-unit partial derivatives of the price (paper section 3,
 * "Greeks"; get_all_greeks returns all five from one d1/d2 evaluation).
 *   delta = dP/dS (BS, BSM) or dP/dF (Black-76)
 *   gamma = d2P/dS2 or d2P/dF2
 *   vega  = dP/dsigma
 *   theta = -dP/dT  (per year)
 *   rho   = dP/dr   (Black-76: at fixed F)                                  */
static void q_greeks(const qin *a, qr sigma, qr out[5])
{
    const int th = a->theta;
    qr d1, d2;
    q_d12(a, sigma, &d1, &d2);
    qr sqT = sqrtq(a->T);
    qr D = q_discount(a);
    qr P = q_price(a, sigma);
    if (a->model == ORC_B76) {
        qr F = a->fs;
        out[0] = th * D * q_Phi(th * d1);
        out[1] = D * q_phi(d1) / (F * sigma * sqT);
        out[2] = D * F * q_phi(d1) * sqT;
        out[3] = a->r * P - D * F * q_phi(d1) * sigma / (2 * sqT);
        out[4] = -a->T * P;
        return;
    }
    qr S = a->fs, qy = q_divyield(a);
    qr Dq = expq(-qy * a->T);
    out[0] = th * Dq * q_Phi(th * d1);
    out[1] = Dq * q_phi(d1) / (S * sigma * sqT);
    out[2] = S * Dq * q_phi(d1) * sqT;
    out[3] = -S * Dq * q_phi(d1) * sigma / (2 * sqT)
             - th * a->r * a->K * D * q_Phi(th * d2)
             + th * qy * S * Dq * q_Phi(th * d1);
    out[4] = th * a->K * a->T * D * q_Phi(th * d2);
}

/* Partial derivatives of the price at fixed sigma with respect to
 * (S or F, K, T, r, q).  Used by the implicit-function gradient. */
static void q_price_partials(const qin *a, qr sigma, qr dP[5])
{
    const int th = a->theta;
    qr g[5];
    q_greeks(a, sigma, g);
    qr d1, d2;
    q_d12(a, sigma, &d1, &d2);
    qr D = q_discount(a);
    dP[0] = g[0];                               /* dP/dS or dP/dF */
    dP[1] = -th * D * q_Phi(th * d2);           /* dP/dK          */
    dP[2] = -g[3];                              /* dP/dT          */
    dP[3] = g[4];                               /* dP/dr          */
    if (a->model == ORC_BSM) {
        qr Dq = expq(-a->q * a->T);
        dP[4] = -th * a->T * a->fs * Dq * q_Phi(th * d1);
    } else {
        dP[4] = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Status decision in binary64                                               */
/* ------------------------------------------------------------------------ */
static int d_status(int model, double price, double fs, double K, double T, double r,
                    double q, int theta)
{
    if (!isfinite(price) || !isfinite(fs) || !isfinite(K) || !isfinite(T) ||
        !isfinite(r) || !isfinite(q))
        return ORC_INVALID;
    if (fs <= 0 || K <= 0 || T <= 0 || (theta != 1 && theta != -1))
        return ORC_INVALID;
    /* the library's input domain: S/F, K and the forward are normal binary64
       numbers (subnormal ones are invalid inputs, not prices) */
    if (fs < DBL_MIN || K < DBL_MIN)
        return ORC_INVALID;
    /* the forward and the undiscounted price correctly rounded to binary64
       (exponents formed in binary128): a binary64 exponent r T would carry
       its own rounding, tens of ulps of F at long maturities */
    double F;
    if (model == ORC_B76)
        F = fs;
    else
        F = (double)((qr)fs * expq((((model == ORC_BSM) ? ((qr)r - (qr)q) : (qr)r)) * (qr)T));
    if (!(F >= DBL_MIN) || !isfinite(F))
        return ORC_INVALID;
    double Pu = (double)((qr)price * expq((qr)r * (qr)T));
    double I = theta > 0 ? (F > K ? F - K : 0.0) : (K > F ? K - F : 0.0);
    double M = theta > 0 ? F : K;
    if (Pu < I) return ORC_BELOW_INTRINSIC;
    if (Pu == I) return ORC_AT_INTRINSIC;
    if (Pu >= M) return ORC_ABOVE_MAX;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The implied volatility: the root of price(sigma) = P, in binary128.       */
/* ------------------------------------------------------------------------ */
/* dP/dsigma = D F phi(d1) sqrt(T)  (for BS/BSM, D F = S e^{-qT}) */
static qr q_vega(const qin *a, qr sigma)
{
    qr d1, d2;
    q_d12(a, sigma, &d1, &d2);
    return q_discount(a) * q_forward(a) * q_phi(d1) * sqrtq(a->T);
}

/* Returns the root; *ok = 0 if no finite positive root exists in exact
 * arithmetic (price on or outside the bounds), *ok = -1 if the iteration
 * hit its cap (never expected; the tests assert it does not happen). */
static qr q_implied_vol(const qin *a, qr P, int *ok)
{
    *ok = 1;
    if (q_price(a, 0) >= P) { *ok = 0; return 0; }
    /* upper bracket: double sigma until the price exceeds P */
    qr lo = 0, hi = 1;
    int k = 0;
    while (q_price(a, hi) < P) {
        lo = hi;
        hi *= 2;
        if (++k > 60) { *ok = 0; return 0; }
    }
    qr sig = (lo > 0) ? 0.5Q * (lo + hi) : 0.5Q * hi;
    /* A Newton step is taken only if it stays inside the bracket and is at
     * most half as long as the step before the previous one; otherwise the
     * bracket is bisected.  So the iterate cannot crawl (Newton from the
     * convex side of a deep out-of-the-money price moves by ~1/h^2 relative
     * per step) and the bracket keeps shrinking. */
    qr step1 = hi, step2 = hi;
    for (int it = 0; it < 4000; ++it) {
        qr f = q_price(a, sig) - P;
        if (f == 0) return sig;
        if (f < 0) lo = sig; else hi = sig;
        qr v = q_vega(a, sig);
        qr nxt = 0;
        int newton_ok = 0;
        if (v > 0) {
            nxt = sig - f / v;
            if (nxt > lo && nxt < hi && fabsq(nxt - sig) <= 0.5Q * step2) newton_ok = 1;
        }
        if (!newton_ok) {
            /* bisection: geometric when the bracket spans more than 4x */
            if (lo > 0 && hi > 4 * lo) nxt = sqrtq(lo * hi);
            else if (lo == 0) nxt = 0.25Q * hi;
            else nxt = 0.5Q * (lo + hi);
        }
        qr step = fabsq(nxt - sig);
        step2 = step1;
        step1 = step;
        sig = nxt;
        if (newton_ok && step <= 1e-31Q * sig) return sig;
        if (hi - lo <= 1e-31Q * hi) return 0.5Q * (lo + hi);
    }
    *ok = -1;
    return sig;
}

static void fill_in(qin *a, int model, double fs, double K, double T, double r, double q,
                    int theta)
{
    a->model = model;
    a->fs = fs;
    a->K = K;
    a->T = T;
    a->r = r;
    a->q = (model == ORC_BSM) ? (qr)q : 0.0Q;
    a->theta = theta;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (arrays of length n, all fields full arrays)        */
/* ------------------------------------------------------------------------ */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* price, rounded to binary64 (hi) with the rounding residual (lo) */
void orc_price_n(int model, int64_t n, const double *fs, const double *K, const double *T,
                 const double *r, const double *q, const double *sigma,
                 const int8_t *flag, double *hi, double *lo)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        qin a;
        fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
        qr p = q_price(&a, sigma[i]);
        double h = (double)p;
        hi[i] = h;
        if (lo) lo[i] = (double)(p - (qr)h);
    }
}

/* five Greeks: delta, gamma, vega, theta, rho (each array of n) */
void orc_greeks_n(int model, int64_t n, const double *fs, const double *K, const double *T,
                  const double *r, const double *q, const double *sigma, const int8_t *flag,
                  double *delta, double *gamma, double *vega, double *theta, double *rho)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        qin a;
        fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
        qr g[5];
        q_greeks(&a, sigma[i], g);
        delta[i] = (double)g[0];
        gamma[i] = (double)g[1];
        vega[i] = (double)g[2];
        theta[i] = (double)g[3];
        rho[i] = (double)g[4];
    }
}

/* Per-quote status only (binary64 decision). */
void orc_status_n(int model, int64_t n, const double *price, const double *fs,
                  const double *K, const double *T, const double *r, const double *q,
                  const int8_t *flag, uint8_t *status)
{
    for (int64_t i = 0; i < n; ++i)
        status[i] = (uint8_t)d_status(model, price[i], fs[i], K[i], T[i], r[i], q[i], flag[i]);
}

/* Implied volatility.  sigma_lo receives the binary128 residual of the root
 * (may be NULL).  Non-OK quotes: NaN, except at intrinsic where sigma = 0. */
void orc_implied_vol_n(int model, int64_t n, const double *price, const double *fs,
                       const double *K, const double *T, const double *r, const double *q,
                       const int8_t *flag, double *sigma, double *sigma_lo, uint8_t *status)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int st = d_status(model, price[i], fs[i], K[i], T[i], r[i], q[i], flag[i]);
        double out = NAN, outlo = 0.0;
        if (st == ORC_AT_INTRINSIC) out = 0.0;
        if (st == ORC_OK) {
            qin a;
            fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
            int ok;
            qr s = q_implied_vol(&a, price[i], &ok);
            if (ok > 0) {
                out = (double)s;
                outlo = (double)(s - (qr)out);
            } else {
                st = ok == 0 ? ORC_NO_EXACT_ROOT : ORC_ROOT_CAP;
            }
        }
        sigma[i] = out;
        if (sigma_lo) sigma_lo[i] = outlo;
        status[i] = (uint8_t)st;
    }
}

/* Gradient of the implied volatility with respect to
 * (price, S or F, K, T, r, q), by the implicit-function theorem at the
 * oracle's own root:  d sigma/d P = 1/vega,
 * d sigma/d X = -(dP/dX at fixed sigma)/vega.
 * grad is row-major [n][6].  Quotes without a root get NaN rows. */
void orc_iv_grad_n(int model, int64_t n, const double *price, const double *fs,
                   const double *K, const double *T, const double *r, const double *q,
                   const int8_t *flag, double *grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double *g = grad + 6 * i;
        for (int j = 0; j < 6; ++j) g[j] = NAN;
        int st = d_status(model, price[i], fs[i], K[i], T[i], r[i], q[i], flag[i]);
        if (st != ORC_OK) continue;
        qin a;
        fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
        int ok;
        qr s = q_implied_vol(&a, price[i], &ok);
        if (ok <= 0) continue;
        qr v = q_vega(&a, s);
        qr dP[5];
        q_price_partials(&a, s, dP);
        g[0] = (double)(1 / v);
        for (int j = 0; j < 5; ++j) g[1 + j] = (double)(-dP[j] / v);
        if (model != ORC_BSM) g[5] = 0.0;
    }
}

/* Signed relative sensitivities of the implied volatility,
 *   e_X = X d sigma/d X   for X in (price, S or F, K, T, r, q),
 * by the implicit-function theorem at the oracle's own root (the gradient
 * above times the input), with the product formed in binary128 before the
 * rounding to binary64.  For prices below the normal binary64 range, vega is
 * far below it as well and 1/vega overflows binary64, while the product
 * X/vega stays of the order of sigma; only this form keeps it finite.
 * rel is row-major [n][6]; quotes without a root get NaN rows.  (r and q
 * enter as absolute values: e_r = r d sigma/d r.) */
void orc_iv_rel_sens_n(int model, int64_t n, const double *price, const double *fs,
                       const double *K, const double *T, const double *r, const double *q,
                       const int8_t *flag, double *rel)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double *e = rel + 6 * i;
        for (int j = 0; j < 6; ++j) e[j] = NAN;
        int st = d_status(model, price[i], fs[i], K[i], T[i], r[i], q[i], flag[i]);
        if (st != ORC_OK) continue;
        qin a;
        fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
        int ok;
        qr s = q_implied_vol(&a, price[i], &ok);
        if (ok <= 0) continue;
        qr v = q_vega(&a, s);
        qr dP[5];
        q_price_partials(&a, s, dP);
        const qr X[5] = {a.fs, a.K, a.T, a.r, a.q};
        e[0] = (double)((qr)price[i] / v);
        for (int j = 0; j < 5; ++j) e[1 + j] = (double)(-dP[j] * X[j] / v);
        if (model != ORC_BSM) e[5] = 0.0;
    }
}

/* The implicit-function gradient formula evaluated at a GIVEN volatility
 * sigma (not at the root): d sigma/d P = 1/vega(sigma),
 * d sigma/d X = -(dP/dX at fixed sigma)/vega(sigma) -- what an adjoint
 * computes from a volatility solved elsewhere.  Rows of NaN where sigma is
 * not finite and positive or the inputs are outside the model's domain;
 * the price does not enter. */
void orc_iv_grad_at_n(int model, int64_t n, const double *fs, const double *K,
                      const double *T, const double *r, const double *q,
                      const double *sigma, const int8_t *flag, double *grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double *row = grad + 6 * i;
        for (int j = 0; j < 6; ++j) row[j] = NAN;
        if (!isfinite(sigma[i]) || !(sigma[i] > 0) || !isfinite(fs[i]) || !isfinite(K[i]) ||
            !isfinite(T[i]) || !(fs[i] > 0) || !(K[i] > 0) || !(T[i] > 0))
            continue;
        qin a;
        fill_in(&a, model, fs[i], K[i], T[i], r[i], q[i], flag[i]);
        qr s = sigma[i];
        qr v = q_vega(&a, s);
        qr dP[5];
        q_price_partials(&a, s, dP);
        row[0] = (double)(1 / v);
        for (int j = 0; j < 5; ++j) row[1 + j] = (double)(-dP[j] / v);
        if (model != ORC_BSM) row[5] = 0.0;
    }
}

/* Normalised Black function b(x, s, theta) =
 *   theta [ e^{x/2} Phi(theta (x/s + s/2)) - e^{-x/2} Phi(theta (x/s - s/2)) ]
 * (normalised coordinates of the paper's section 1: x = ln(F/K), s = sigma
 * sqrt(T); price = D sqrt(F K) b).  hi/lo as for orc_price_n. */
void orc_normalised_black_n(int64_t n, const double *x, const double *s, const int8_t *flag,
                            double *hi, double *lo)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        qr X = x[i], S = s[i];
        int th = flag[i];
        qr b;
        if (S <= 0) {
            qr iv = th * (expq(X / 2) - expq(-X / 2));
            b = iv > 0 ? iv : 0;
        } else {
            qr h = X / S, t = S / 2;
            b = th * (expq(X / 2) * q_Phi(th * (h + t)) - expq(-X / 2) * q_Phi(th * (h - t)));
        }
        double d = (double)b;
        hi[i] = d;
        if (lo) lo[i] = (double)(b - (qr)d);
    }
}
