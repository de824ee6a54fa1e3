/*
 * fastvol.h -- C ABI of the MI355X (gfx950) batched implied-volatility library.
 *
 * European options under Black-76, Black-Scholes and Black-Scholes-Merton
 * (the three models of the paper's section 3, "Capabilities"): pricing,
 * implied volatility with the "Let's Be Rational" solver or the Halley
 * solver (section 2.2, "Dual-Solver Design"), the five Greeks (section 3,
 * get_all_greeks), the implicit-function gradient of the implied volatility
 * (section 3, "Differentiable IV") and ragged option chains in one launch.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers (e.g. torch.Tensor.data_ptr() of a
 *    CUDA/HIP tensor) owned by the caller.  The library never allocates,
 *    frees or retains them; a call may be captured into a hipGraph, in which
 *    case the caller keeps the buffers alive for the graph's lifetime.
 *  - Float arrays are IEEE binary64, contiguous, one element per quote
 *    (struct-of-arrays).  Flags are int8: +1 call, -1 put.
 *  - fv_arg: a per-quote field is either an array (ptr != NULL) or one value
 *    broadcast to every quote (ptr == NULL, `value` used) -- the paper's
 *    broadcastable inputs (section 2.1).
 *  - `stream` is a hipStream_t cast to void* (NULL = the null stream).  Every
 *    call only enqueues work and returns; nothing synchronises the host.
 *  - Return value: FV_OK, or a negative fv_status when the call itself is
 *    invalid (nothing is launched; fv_last_error() says why).  n == 0 is a
 *    no-op returning FV_OK; n above (2^31 - 1) * 64 (more workgroups than a
 *    launch can have) is FV_E_INVALID_ARG.  Per-quote problems never fail a call: they are
 *    reported in the per-quote status array (fv_quote_status).
 *  - Black-76 prices are DISCOUNTED (section 2.4): price = e^{-rT} Black(F).
 *    T is in years; r, q continuously compounded.
 *  - Greeks are raw per-unit partial derivatives: delta = dP/dS (dP/dF for
 *    Black-76), gamma = d2P/dS2, vega = dP/dsigma, theta = -dP/dT per year,
 *    rho = dP/dr (Black-76: at fixed F).
 *  - Not thread-safe across concurrent calls that share output buffers;
 *    otherwise calls from several host threads are independent, except that
 *    fv_set_launch, fv_autotune and fv_set_halley_steps change process-wide
 *    settings and must not run while another thread launches.
 */
#ifndef FASTVOL_H
#define FASTVOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FV_ABI_VERSION 1

typedef enum {
    FV_MODEL_BLACK76 = 0,        /* forward F, discounted price            */
    FV_MODEL_BLACK_SCHOLES = 1,  /* spot S, no dividend yield (q ignored)  */
    FV_MODEL_BSM = 2             /* spot S, continuous dividend yield q    */
} fv_model;

typedef enum {
    FV_SOLVER_LBR = 0,     /* rational guess + Householder(3): reference grade */
    FV_SOLVER_HALLEY = 1   /* Halley (<= 8 steps) + bisection fallback        */
} fv_solver;

typedef enum {
    FV_OK = 0,
    FV_E_INVALID_ARG = -1,  /* NULL required pointer, n < 0, bad enum, bad size */
    FV_E_HIP = -2,          /* the HIP runtime refused a launch                 */
    FV_E_UNSUPPORTED = -3   /* e.g. no gfx950 device                            */
} fv_status;

/* per-quote status codes (uint8 arrays) */
enum fv_quote_status {
    FV_Q_OK = 0,
    FV_Q_AT_INTRINSIC = 1,     /* undiscounted price == intrinsic: sigma = 0    */
    FV_Q_BELOW_INTRINSIC = 2,  /* price below intrinsic: sigma = NaN            */
    FV_Q_ABOVE_MAX = 3,        /* price >= the no-arbitrage maximum: NaN        */
    FV_Q_INVALID_INPUT = 4,    /* non-finite input, S/F, K or T <= 0, bad flag;
                                  for the implied-volatility entry points also
                                  S/F, K or the forward below the smallest
                                  normal number (or the forward overflowing) */
    FV_Q_NOT_CONVERGED = 5     /* solver did not meet its tolerance, or its root was
                                  not finite and positive (sigma keeps the last
                                  iterate; NaN on the binary32 path) */
};

typedef struct {
    const double *ptr;  /* device array of n values, or NULL to broadcast `value` */
    double value;
} fv_arg;

/* A flat batch of n quotes.  `fs` is F for Black-76 and S otherwise.  `q` is
 * read only for FV_MODEL_BSM.  `price` is read only by the implied-volatility
 * entry points.  flag: device int8 array of +1/-1, or NULL to broadcast
 * flag_value. */
typedef struct {
    int64_t n;
    fv_arg price, fs, K, T, r, q;
    const int8_t *flag;
    int8_t flag_value;
} fv_quotes;

/* Ragged Black-76 option chains in CSR form (one persistent launch):
 * chain c owns maturities chain_mat_off[c] .. chain_mat_off[c+1]-1, maturity m
 * owns quotes mat_quote_off[m] .. mat_quote_off[m+1]-1.  F and r are per
 * chain, T per maturity; price, K, flag per quote.  Offsets are int64,
 * non-decreasing, chain_mat_off[0] = mat_quote_off[0] = 0,
 * chain_mat_off[n_chains] = n_maturities, mat_quote_off[n_maturities] =
 * n_quotes.  All arrays are device arrays. */
typedef struct {
    int64_t n_chains, n_maturities, n_quotes;
    const int64_t *chain_mat_off;  /* [n_chains + 1]     */
    const int64_t *mat_quote_off;  /* [n_maturities + 1] */
    const double *F;               /* [n_chains]         */
    const double *r;               /* [n_chains]         */
    const double *T;               /* [n_maturities]     */
    const double *price;           /* [n_quotes] discounted Black-76 prices */
    const double *K;               /* [n_quotes]         */
    const int8_t *flag;            /* [n_quotes]         */
} fv_chains;

/* Model price at volatility sigma (paper section 3: fast_black,
 * fast_black_scholes, fast_black_scholes_merton).  Evaluated through the
 * normalised Black function, so deep out-of-the-money prices keep their
 * relative precision.  q->price is ignored.  Inputs outside the domain
 * (non-finite, S/F, K, T <= 0, sigma < 0) give NaN. */
int fv_price(int model, const fv_quotes *q, fv_arg sigma, double *price_out, void *stream);

/* Implied volatility (paper sections 1 and 2.2): the sigma >= 0 at which the
 * model price equals q->price.  solver = FV_SOLVER_LBR or FV_SOLVER_HALLEY.
 * sigma_out: [n] (required).  status_out: [n] uint8 or NULL.
 * greeks_out: NULL, or an array of 5 pointers (delta, gamma, vega, theta,
 * rho), each [n] or NULL, filled at the solved sigma in the same pass (NaN
 * where the status is not FV_Q_OK). */
int fv_implied_vol(int model, int solver, const fv_quotes *q, double *sigma_out,
                   uint8_t *status_out, double *const *greeks_out, void *stream);

/* A flat batch in binary32: the layout of fv_quotes with float fields. */
typedef struct {
    const float *ptr;  /* device array of n values, or NULL to broadcast `value` */
    float value;
} fv_arg_f32;

typedef struct {
    int64_t n;
    fv_arg_f32 price, fs, K, T, r, q;
    const int8_t *flag;
    int8_t flag_value;
} fv_quotes_f32;

/* Implied volatility in binary32 arithmetic with the Halley path (paper
 * section 2.2: the throughput solver for label pipelines that train in
 * float32): Brenner-Subrahmanyam start, at most 8 Halley steps (the
 * fv_set_halley_steps limit), bisection for the quotes that fail the
 * convergence check, all in float.
 * sigma_out: float [n] (required); status_out: uint8 [n] or NULL.  Statuses
 * as for fv_implied_vol; FV_Q_NOT_CONVERGED (sigma NaN) also marks a quote
 * whose normalised out-of-the-money price beta = P_undiscounted/sqrt(F K)
 * (less the intrinsic value) is below 2^-100, outside this solver's domain
 * (the binary64 entry points solve it).  Accuracy: |sigma - sigma*| <=
 * max(4e-6 sigma*, 8 u32 sum_X |d sigma/d X| |X|) against the exact root
 * sigma* of the given binary32 inputs, u32 = 2^-24 (the second term is the
 * sensitivity of the root to rounding its inputs). */
int fv_implied_vol_f32(int model, const fv_quotes_f32 *q, float *sigma_out, uint8_t *status_out,
                       void *stream);

/* The five Greeks at volatility sigma (paper section 3, get_all_greeks).
 * Each output [n] may be NULL.  q->price is ignored. */
int fv_greeks(int model, const fv_quotes *q, fv_arg sigma, double *delta, double *gamma,
              double *vega, double *theta, double *rho, void *stream);

/* Adjoint of fv_implied_vol (paper section 3, "Differentiable IV"), by the
 * implicit-function theorem: dsigma/dP = 1/vega and
 * dsigma/dX = -(dP/dX at fixed sigma)/vega for X in (S or F, K, T, r, q).
 * sigma: [n] solved volatilities; grad_sigma: [n] upstream gradient dL/dsigma.
 * Outputs dL/dX = grad_sigma * dsigma/dX, each [n] or NULL.  Quotes whose
 * sigma is not finite and positive get zero gradients.  g_q is zero for
 * Black-76 and Black-Scholes. */
int fv_implied_vol_backward(int model, const fv_quotes *q, const double *sigma,
                            const double *grad_sigma, double *g_price, double *g_fs,
                            double *g_K, double *g_T, double *g_r, double *g_q, void *stream);

/* Adjoint of fv_price: from the upstream gradient grad_price = dL/dP [n],
 * dL/dX = grad_price * dP/dX at fixed inputs for X in (S or F, K, T, r, q,
 * sigma): delta, -theta D Phi(theta d2), -(Greek theta), rho,
 * -theta T D F Phi(theta d1) (Black-Scholes-Merton; 0 otherwise), vega.
 * Each output [n] may be NULL.  Quotes outside the pricing domain or with
 * sigma <= 0 get zeros.  q->price is ignored. */
int fv_price_backward(int model, const fv_quotes *q, fv_arg sigma, const double *grad_price,
                      double *g_fs, double *g_K, double *g_T, double *g_r, double *g_q,
                      double *g_sigma, void *stream);

/* Implied volatility of ragged Black-76 chains in ONE launch over the flat
 * quote range: one workgroup per fixed-size chunk of consecutive quotes (the
 * hardware scheduler balances the uneven per-quote cost; no grid-stride
 * loop), each wave finding its quotes' maturity and chain through the CSR
 * offsets, so no per-quote F, r or T array is materialised.
 * sigma_out [n_quotes] required, status_out [n_quotes] or NULL. */
int fv_implied_vol_chains(int solver, const fv_chains *c, double *sigma_out,
                          uint8_t *status_out, void *stream);

/* Calibration problem: per-maturity SVI smiles on ragged Black-76 chains,
 * fitted through the differentiable implied volatility (the paper's
 * section 1 motivation -- IV inside calibration pipelines -- with the
 * autograd-friendly IV of section 3).  Per maturity m the raw parameters are
 * theta[5m .. 5m+4] = (a, b~, rho~, mu, s~) with b = softplus(b~),
 * rho = tanh(rho~), s = softplus(s~), total variance
 *   w(k) = a + b (rho (k - mu) + sqrt((k - mu)^2 + s^2)),  k = ln(K/F),
 * sigma_SVI = sqrt(w/T).  The loss is
 *   L = (1/n_quotes) sum_i (IV(P_Black76(sigma_SVI,i)) - iv_target_i)^2,
 * quotes with w <= 1e-10 or a non-finite target contribute nothing; where
 * the model price of sigma_SVI is not solvable in binary64 (its normalised
 * value rounded onto 0 or onto its upper bound) IV(P(sigma_SVI)) takes its
 * exact value sigma_SVI.  chains.price is not read; all arrays are device
 * arrays. */
typedef struct {
    fv_chains chains;
    const double *iv_target;             /* [n_quotes] */
    double lr, beta1, beta2, eps;        /* Adam hyper-parameters */
} fv_svi_problem;

/* Size in doubles of the workspace fv_svi_adam_step needs for problem p:
 * 2 + 8 n_maturities + ceil(n_maturities / 4)
 *   + 6 (ceil(n_quotes / 64) + n_maturities).
 * Negative (an FV_E_* code) when p is invalid. */
int64_t fv_svi_workspace_size(const fv_svi_problem *p);

/* One Adam step of the calibration, as four launches on `stream` that
 * allocate nothing and never synchronise (capturable in a hipGraph): the
 * per-maturity natural parameters; the per-quote chain SVI -> Black-76
 * price -> LBR implied volatility -> implicit-function adjoint, one wave per
 * 64 consecutive quotes, summed per (wave, maturity) run; per maturity the
 * sums of its runs in a fixed order, the gradient and the Adam update; the
 * loss, a fixed-order sum (not launched when loss is NULL or loss_len is
 * 0).  No atomics: results are bitwise reproducible.  The price reaches the
 * solver as the normalised price b(x, s) of its out-of-the-money side, the
 * value the solver's own reduction of the discounted price recovers.
 *   theta, adam_m, adam_v: [5 n_maturities] in/out (moments start at 0);
 *   step: one device int64 (Adam's step count t, read then incremented);
 *   grad: [5 n_maturities] out: gradient at the pre-update theta;
 *   workspace: device scratch of workspace_len >= fv_svi_workspace_size(p)
 *   doubles (FV_E_INVALID_ARG if smaller); the step writes every value it
 *   reads there before reading it, so its contents between calls do not
 *   matter; steps that share a workspace must not overlap in time;
 *   loss: [loss_len] history (may be NULL): loss[t] receives the loss at the
 *   pre-update theta of step t (t read from *step; nothing written when
 *   t >= loss_len).  A replayed graph thus records every step's loss. */
int fv_svi_adam_step(const fv_svi_problem *p, double *theta, double *adam_m, double *adam_v,
                     int64_t *step, double *grad, double *workspace, int64_t workspace_len,
                     double *loss, int64_t loss_len, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as fv_svi_adam_step, with its workspace taken from an array the
 * library holds on each GPU (8 MiB, 1,048,576 doubles, kept until the
 * process ends) instead of a caller buffer.  Problems whose
 * fv_svi_workspace_size exceeds that get FV_E_INVALID_ARG and launch
 * nothing.  Nothing is allocated: the array is part of the loaded code
 * object, and its address is looked up once per device (on the first call
 * with that device current).  Every call on one GPU shares that GPU's
 * array, so calls that overlap in time on one GPU (two streams, two host
 * threads) race and must be serialised by the caller.  The step writes
 * every workspace value it reads before reading it, so what an earlier call
 * left there does not matter. */
int fv_svi_adam_step_noalloc(const fv_svi_problem *p, double *theta, double *adam_m,
                             double *adam_v, int64_t *step, double *grad, double *loss,
                             int64_t loss_len, void *stream);

/* sigma_SVI of every quote at parameters theta [5 n_maturities];
 * sigma_out [n_quotes] (NaN where w <= 0). */
int fv_svi_vols(const fv_svi_problem *p, const double *theta, double *sigma_out, void *stream);

/* Normalised Black function b(x, s, theta) (the evaluator underneath every
 * entry point): theta [e^{x/2} Phi(theta(x/s + s/2)) - e^{-x/2}
 * Phi(theta(x/s - s/2))].  x, s: device arrays [n] (s >= 0); flag: device
 * int8 [n] or NULL for calls.  out: [n].  Out of the money the result is
 * within a few ulps of the exact b at the given x and s (the exponent
 * -(x^2/s^2 + s^2/4)/2 is formed to twice the working precision), and below
 * the normal range within a few units of the smallest subnormal. */
int fv_normalised_black(int64_t n, const double *x, const double *s, const int8_t *flag,
                        double *out, void *stream);

/* Diagnostic: the path each quote takes through the LBR solver, as
 * fv_implied_vol(..., FV_SOLVER_LBR, ...) solves it.  path_out: uint32 [n];
 * bits 0-1 guess region (0..3 = lower map / lower interior / upper interior /
 * upper map), bits 2-3 Householder(3) steps minus 2, bits 4-5 and 6-7 the
 * normalised-Black evaluation form at the two boundary points, from bit 8
 * two bits per step (forms: 0 divided difference of erfcx, 1 complement
 * b_max - b).  0xFFFFFFFF for quotes whose status is not FV_Q_OK.  Used to
 * group quotes by path, e.g. to measure divergence. */
int fv_lbr_trace(int model, const fv_quotes *q, uint32_t *path_out, void *stream);

/* Diagnostic: the Halley steps each quote takes as fv_implied_vol(...,
 * FV_SOLVER_HALLEY, ...) solves it (paper section 2.2, the throughput path).
 * steps_out: uint32 [n]; bits 0-7 the number of Halley steps (1 up to the
 * fv_set_halley_steps limit, 8 by default), bit 8 set when the quote fails
 * the convergence check and goes through the bisection fallback; 0xFFFFFFFF
 * for quotes whose status is not FV_Q_OK.  Used to group quotes by work,
 * e.g. to measure divergence. */
int fv_halley_trace(int model, const fv_quotes *q, uint32_t *steps_out, void *stream);

/* The Halley path's step limit (paper section 2.2: a fixed number of Halley
 * steps, then bisection for the quotes that fail the convergence check).
 * Every Halley launch (fv_implied_vol with FV_SOLVER_HALLEY, the ragged
 * chains, fv_implied_vol_f32, fv_halley_trace) reads it when it is
 * enqueued; default 8.  In binary64 the iteration starts from the LBR
 * path's initial guess and its first step is at guess precision, so a quote
 * never stops before its second step: a limit of 1 sends every solvable
 * quote to the fallback, 2 the quotes that need a third step (binary32
 * starts from the Brenner-Subrahmanyam form and may stop after any step).
 * Results stay within the Halley tolerance at any
 * limit (the fallback bisects to 1e-13 relative); a lower limit only moves
 * work to the slower bisection, which makes it a way to exercise that path.
 * steps in [1, 64], FV_E_INVALID_ARG otherwise (the limit in force is
 * kept).  Process-wide, like fv_set_launch. */
int fv_set_halley_steps(int steps);
int fv_get_halley_steps(void);

/* Launch-shape control.  fv_set_launch(kernel, block, quotes_per_thread)
 * overrides the launch shape of one kernel family (FV_KERNEL_*); block must
 * be a multiple of 64 in [64, 512] and quotes_per_thread in [1, 16], and for
 * the Halley families the workgroup's queue of unconverged quotes (24 bytes
 * per quote, 16 for binary32; the ragged-chain kernel, which takes two
 * 64-quote slices per wave and ignores quotes_per_thread, 64 bytes per
 * thread) must fit in 64 KiB of LDS
 * (FV_E_INVALID_ARG otherwise; the shape in force is kept).
 * fv_get_launch reads the configured shape.  The shape applies as set to
 * batches large enough to fill the device; a batch that would give fewer
 * than 8 waves per SIMD (32 per compute unit) runs with fewer quotes per
 * thread (halved until it has them, or one per thread), and with fewer than
 * one workgroup per compute unit also with 64-thread workgroups.  No result
 * depends on the
 * shape.
 *
 * Autotuner: fv_autotune(kernel, model, n_hint, stream) times the candidate
 * shapes (block 64..512, 1..8 quotes per thread, within the LDS limit above)
 * of one kernel family on `stream` with synthetic in-range quotes, on a
 * batch of min(n_hint, 2^24) quotes (whole groups of 2,048), and keeps the
 * fastest for that family, model and the size class of n_hint -- the
 * classes are n < 2^14, [2^14, 2^16), [2^16, 2^18), [2^18, 2^20),
 * [2^20, 2^22), [2^22, 2^24) and n >= 2^24 (the ragged family is always
 * Black-76).  From then on a launch whose batch falls in a tuned class uses
 * the tuned shape as measured; untuned classes keep the configured shape and
 * its narrowing.  fv_autotune allocates and frees scratch for this call only
 * and synchronises the stream: it is not graph-capturable.  fv_set_launch
 * clears the family's tuned classes (an explicit shape wins).
 * fv_launch_shape reports the shape a launch of n >= 1 quotes would use.
 * fv_tuning_save writes every tuned class to a JSON file stamped with the
 * device's architecture name (hipDeviceProp_t::gcnArchName);
 * fv_tuning_load replaces the tuned classes with a file's, validating every
 * entry first (FV_E_INVALID_ARG for an unreadable or malformed file, nothing
 * applied) and refusing a file written on another architecture
 * (FV_E_UNSUPPORTED); fv_tuning_reset forgets every tuned class.  These
 * calls change process-wide state (see the threading note above). */
enum fv_kernel {
    FV_KERNEL_PRICE = 0,
    FV_KERNEL_IV_LBR = 1,
    FV_KERNEL_IV_HALLEY = 2,
    FV_KERNEL_GREEKS = 3,
    FV_KERNEL_BACKWARD = 4,
    FV_KERNEL_CHAINS = 5,
    FV_KERNEL_IV_HALLEY_F32 = 6,
    FV_KERNEL_COUNT = 7
};
int fv_set_launch(int kernel, int block, int quotes_per_thread);
int fv_get_launch(int kernel, int *block, int *quotes_per_thread);
int fv_autotune(int kernel, int model, int64_t n_hint, void *stream);
int fv_launch_shape(int kernel, int model, int64_t n, int *block, int *quotes_per_thread);
int fv_tuning_reset(void);
int fv_tuning_save(const char *path);
int fv_tuning_load(const char *path);

/* Human-readable reason of the last failed call on this host thread. */
const char *fv_last_error(void);
/* FV_ABI_VERSION of the loaded library. */
int fv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTVOL_H */
