// fv_calib.hip -- calibration of per-maturity SVI smiles on ragged Black-76
// chains through the differentiable implied volatility (the paper's use
// case of IV "inside differentiable pipelines for calibration", section 1,
// with the autograd-friendly IV of section 3).
//
// Model per maturity, raw parameters theta = (a, b~, rho~, m, s~):
//   b = softplus(b~), rho = tanh(rho~), s = softplus(s~),
//   w(k) = a + b (rho (k - m) + sqrt((k - m)^2 + s^2)),   k = ln(K/F),
//   sigma_SVI = sqrt(w / T).
// Loss over the N quotes: L = (1/N) sum (IV(P_B76(sigma_SVI)) - IV_target)^2.
// One step = two launches, both graph-capturable (no allocation, no host
// synchronisation, no memset):
//   1. one workgroup per maturity: for each quote, SVI -> Black-76 price ->
//      LBR implied volatility -> residual -> adjoint (dIV/dP = 1/vega(IV),
//      dP/dsigma = vega(sigma), dsigma/dw = 1/(2 sigma T), dw/dtheta), summed
//      over the maturity's quotes in registers and then in LDS in a fixed
//      order (deterministic, no atomics); its first thread also advances the
//      step counter;
//   2. Adam update of every parameter with the advanced counter; its first
//      workgroup also sums the per-maturity losses in a fixed order.
// The price is handed to the solver in the normalised coordinates it
// reduces every quote to: the Black-76 price of the model is
// D sqrt(F K) (b(x, s) + intrinsic), and the solver's reduction (undiscount,
// subtract the intrinsic value, divide by sqrt(F K)) takes it back to
// beta = b(x, s) exactly in exact arithmetic, so the kernel passes beta = b
// of the out-of-the-money side to the LBR solve without the round trip.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/fastvol.h"
#include "fv_host.h"
#include "fv_quote.h"

namespace {

constexpr int kCalibBlock = 256;
constexpr double kWMin = 1e-10;  // total variance floor: quotes below it are skipped

struct KSvi {
  int64_t n_chains, n_mat, n;
  const int64_t* chain_mat_off;
  const int64_t* mat_quote_off;
  const double *F, *r, *T, *K;
  const int8_t* flag;
  const double* iv_target;
};

__device__ __forceinline__ double softplus(double z) { return z > 30.0 ? z : log1p(exp(z)); }
__device__ __forceinline__ double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

// Per-maturity constants of the raw parametrisation.
struct SviMat {
  double a, b, rho, m, s2, sb, ss;  // sb, ss: softplus' of b~ and s~ (sigmoids)
  double s;
};

__device__ __forceinline__ SviMat svi_mat(const double* th) {
  SviMat q;
  q.a = th[0];
  q.b = softplus(th[1]);
  q.rho = tanh(th[2]);
  q.m = th[3];
  q.s = softplus(th[4]);
  q.s2 = q.s * q.s;
  q.sb = sigmoid(th[1]);
  q.ss = sigmoid(th[4]);
  return q;
}

// total variance at log-moneyness k
__device__ __forceinline__ double svi_w(const SviMat& q, double k) {
  const double dk = k - q.m;
  return q.a + q.b * (q.rho * dk + sqrt(dk * dk + q.s2));
}

// sqrt((k - m)^2 + s^2) and its reciprocal, shared by w and dw/dtheta; the
// refined hardware reciprocal square root where the radicand is a normal
// number, the library square root otherwise (s underflowed to 0 at k = m)
struct SviRoot {
  double dk, rt, irt;
};

__device__ __forceinline__ SviRoot svi_root(const SviMat& q, double k) {
  SviRoot o;
  o.dk = k - q.m;
  const double u = fma(o.dk, o.dk, q.s2);
  if (u >= 2.2250738585072014e-308) {
    o.irt = fv::rsqrt(u);
    o.rt = u * o.irt;
  } else {
    o.rt = sqrt(u);
    o.irt = 1.0 / o.rt;
  }
  return o;
}

// g_w * dw/dtheta added into acc[0..4]
__device__ __forceinline__ void svi_add_grad(const SviMat& q, const SviRoot& g, double g_w,
                                             double* acc) {
  const double dk = g.dk, rt = g.rt, irt = g.irt;
  acc[0] += g_w;
  acc[1] += g_w * (q.rho * dk + rt) * q.sb;
  acc[2] += g_w * q.b * dk * (1.0 - q.rho * q.rho);
  acc[3] += g_w * q.b * (-q.rho - dk * irt);
  acc[4] += g_w * q.b * (q.s * irt) * q.ss;
}

// Largest c in [0, n_chains) with chain_mat_off[c] <= m.
__device__ __forceinline__ int64_t chain_of(const int64_t* off, int64_t n_chains, int64_t m) {
  int64_t lo = 0, hi = n_chains;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= m) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kCalibBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_svi_grad(
    KSvi c, const double* __restrict__ theta,
                                                          double* __restrict__ grad,
                                                          double* __restrict__ loss_parts,
                                                          int64_t* __restrict__ step) {
  __shared__ double red[6][kCalibBlock];
  const int64_t m = blockIdx.x;
  const int64_t ch = chain_of(c.chain_mat_off, c.n_chains, m);
  const double F = c.F[ch], T = c.T[m];
  const double sqT = sqrt(T), iT = 1.0 / T, isqT = 1.0 / sqT;
  double th[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) th[j] = theta[m * 5 + j];
  const SviMat q = svi_mat(th);
  const double inv_n = 1.0 / (double)c.n;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = c.mat_quote_off[m] + threadIdx.x; i < c.mat_quote_off[m + 1];
       i += blockDim.x) {
    const double tgt = c.iv_target[i];
    const double lfk = fv::flog(F * fv::rcp(c.K[i]));  // ln(F/K) = -k
    const SviRoot g = svi_root(q, -lfk);
    const double w = fma(q.b, fma(q.rho, g.dk, g.rt), q.a);
    if (!(w > kWMin) || !fv::finite_d(tgt)) continue;
    const double v = w * iT;
    const double sigma = v * fv::rsqrt(v);
    const double s1 = sigma * sqT;
    // out-of-the-money side: x <= 0, beta = b(x, s1)
    const double x = -fabs(lfk);
    const double bmax = fv::fexp(0.5 * x);
    const fv::NBlack nb = fv::normalised_black(x, s1, bmax);
    // IV(P(sigma)) through the LBR solver; where the model price is not
    // solvable in binary64 (b rounded onto 0 or onto its bound b_max) the
    // composite takes its exact value sigma and unit slope
    double iv = sigma, ratio = 1.0;
    if (nb.b > 0.0 && nb.b < bmax) {
      // ln beta from the evaluator's logarithmic parts (accurate also where
      // b is below the normal range)
      const double ln_beta = nb.lnbp + fv::flog(nb.ratio);
      const fv::LbrResult res = fv::lbr_solve(x, nb.b, bmax, ln_beta, 2, 4, 1e-6);
      iv = res.s * isqT;
      // vega(v) = D F phi(d1(v)) sqrt(T); only vega(sigma)/vega(iv) enters
      const double s2 = res.s;
      const double d1a = fma(lfk, fv::rcp(s1), 0.5 * s1), d1b = fma(lfk, fv::rcp(s2), 0.5 * s2);
      ratio = fv::fexp(-0.5 * (d1a - d1b) * (d1a + d1b));
    }
    const double e = iv - tgt;
    const double g_w = e * inv_n * ratio * fv::rcp(sigma * T);  // (2 e/N) ratio / (2 sigma T)
    svi_add_grad(q, g, g_w, acc);
    acc[5] += e * e;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int wd = kCalibBlock / 2; wd > 0; wd >>= 1) {
    if ((int)threadIdx.x < wd) {
#pragma unroll
      for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + wd];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 5; ++j) grad[m * 5 + j] = red[j][0];
    loss_parts[m] = red[5][0];
    // no other workgroup of this launch reads the counter
    if (m == 0) *step += 1;
  }
}

// Adam with the counter k_svi_grad advanced (t = step, bias corrections
// 1 - beta^t); workgroup 0 also writes loss[t - 1], the fixed-order sum of
// the per-maturity losses over N.
__global__ __launch_bounds__(kCalibBlock) void k_svi_adam(
    int64_t n_par, double* __restrict__ theta, double* __restrict__ am, double* __restrict__ av,
    const double* __restrict__ grad, const int64_t* __restrict__ step, double lr, double b1,
    double b2, double eps, int64_t n_mat, int64_t n, const double* __restrict__ parts,
    double* __restrict__ loss, int64_t loss_len) {
  const int64_t t = *step;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_par) {
    const double g = grad[j];
    const double mo = b1 * am[j] + (1.0 - b1) * g;
    const double v = b2 * av[j] + (1.0 - b2) * g * g;
    am[j] = mo;
    av[j] = v;
    const double mh = mo / (1.0 - pow(b1, (double)t));
    const double vh = v / (1.0 - pow(b2, (double)t));
    theta[j] -= lr * mh / (sqrt(vh) + eps);
  }
  if (blockIdx.x != 0) return;
  __shared__ double red[kCalibBlock];
  double a = 0.0;
  for (int64_t mm = threadIdx.x; mm < n_mat; mm += blockDim.x) a += parts[mm];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int wd = kCalibBlock / 2; wd > 0; wd >>= 1) {
    if ((int)threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss && t >= 1 && t <= loss_len) loss[t - 1] = red[0] / (double)n;
}

__global__ void k_svi_vols(KSvi c, const double* __restrict__ theta, double* __restrict__ out) {
  const int64_t m = blockIdx.x;
  const double T = c.T[m];
  const int64_t ch = chain_of(c.chain_mat_off, c.n_chains, m);
  const double F = c.F[ch];
  double th[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) th[j] = theta[m * 5 + j];
  const SviMat q = svi_mat(th);
  for (int64_t i = c.mat_quote_off[m] + threadIdx.x; i < c.mat_quote_off[m + 1];
       i += blockDim.x) {
    const double w = svi_w(q, log(c.K[i] / F));
    out[i] = w > 0.0 ? sqrt(w / T) : __builtin_nan("");
  }
}

int check_problem(const fv_svi_problem* p) {
  if (!p) return fvh::fail(FV_E_INVALID_ARG, "problem pointer is NULL");
  const fv_chains& c = p->chains;
  if (c.n_chains <= 0 || c.n_maturities <= 0 || c.n_quotes <= 0)
    return fvh::fail(FV_E_INVALID_ARG, "empty or negative chain sizes");
  if (c.n_maturities > 0x7fffffff) return fvh::fail(FV_E_INVALID_ARG, "too many maturities");
  if (!c.chain_mat_off || !c.mat_quote_off || !c.F || !c.r || !c.T || !c.K || !c.flag)
    return fvh::fail(FV_E_INVALID_ARG, "NULL chain array");
  return FV_OK;
}

KSvi to_k(const fv_svi_problem* p) {
  KSvi k;
  const fv_chains& c = p->chains;
  k.n_chains = c.n_chains;
  k.n_mat = c.n_maturities;
  k.n = c.n_quotes;
  k.chain_mat_off = c.chain_mat_off;
  k.mat_quote_off = c.mat_quote_off;
  k.F = c.F;
  k.r = c.r;
  k.T = c.T;
  k.K = c.K;
  k.flag = c.flag;
  k.iv_target = p->iv_target;
  return k;
}

}  // namespace

extern "C" {

int fv_svi_adam_step(const fv_svi_problem* p, double* theta, double* adam_m, double* adam_v,
                     int64_t* step, double* grad, double* loss_parts, double* loss,
                     int64_t loss_len, void* stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (!p->iv_target || !theta || !adam_m || !adam_v || !step || !grad || !loss_parts)
    return fvh::fail(FV_E_INVALID_ARG, "NULL parameter, state or scratch array");
  if (loss_len < 0) return fvh::fail(FV_E_INVALID_ARG, "loss_len < 0");
  if (!(p->lr > 0.0) || !(p->beta1 >= 0.0 && p->beta1 < 1.0) ||
      !(p->beta2 >= 0.0 && p->beta2 < 1.0) || !(p->eps > 0.0))
    return fvh::fail(FV_E_INVALID_ARG, "Adam hyper-parameters out of range");
  const KSvi k = to_k(p);
  hipStream_t s = (hipStream_t)stream;
  k_svi_grad<<<dim3((unsigned)k.n_mat), dim3(kCalibBlock), 0, s>>>(k, theta, grad, loss_parts,
                                                                   step);
  const int64_t n_par = 5 * k.n_mat;
  k_svi_adam<<<dim3((unsigned)((n_par + kCalibBlock - 1) / kCalibBlock)), dim3(kCalibBlock), 0, s>>>(
      n_par, theta, adam_m, adam_v, grad, step, p->lr, p->beta1, p->beta2, p->eps, k.n_mat, k.n,
      loss_parts, loss, loss_len);
  return fvh::launched("fv_svi_adam_step");
}

int fv_svi_vols(const fv_svi_problem* p, const double* theta, double* sigma_out, void* stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (!theta || !sigma_out) return fvh::fail(FV_E_INVALID_ARG, "NULL theta or output");
  const KSvi k = to_k(p);
  k_svi_vols<<<dim3((unsigned)k.n_mat), dim3(kCalibBlock), 0, (hipStream_t)stream>>>(k, theta,
                                                                                    sigma_out);
  return fvh::launched("fv_svi_vols");
}

}  // extern "C"
