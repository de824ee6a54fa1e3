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
// One step = three launches, all graph-capturable (no allocation, no host
// synchronisation, no memset):
//   1. one workgroup per maturity: for each quote, SVI -> Black-76 price ->
//      LBR implied volatility -> residual -> adjoint (dIV/dP = 1/vega(IV),
//      dP/dsigma = vega(sigma), dsigma/dw = 1/(2 sigma T), dw/dtheta), summed
//      over the maturity's quotes in registers and then in LDS in a fixed
//      order (deterministic, no atomics);
//   2. Adam update of every parameter;
//   3. deterministic sum of the per-maturity losses and step += 1.
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

struct SviPoint {
  double w, dw[5];  // total variance and its gradient in the raw parameters
};

__device__ __forceinline__ SviPoint svi_eval(const double* th, double k) {
  const double a = th[0], b = softplus(th[1]), rho = tanh(th[2]), m = th[3],
               s = softplus(th[4]);
  const double dk = k - m;
  const double rt = sqrt(dk * dk + s * s);
  SviPoint p;
  p.w = a + b * (rho * dk + rt);
  p.dw[0] = 1.0;
  p.dw[1] = (rho * dk + rt) * sigmoid(th[1]);
  p.dw[2] = b * dk * (1.0 - rho * rho);
  p.dw[3] = b * (-rho - dk / rt);
  p.dw[4] = b * (s / rt) * sigmoid(th[4]);
  return p;
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

__global__ __launch_bounds__(kCalibBlock) void k_svi_grad(KSvi c, const double* __restrict__ theta,
                                                          double* __restrict__ grad,
                                                          double* __restrict__ loss_parts) {
  __shared__ double red[6][kCalibBlock];
  const int64_t m = blockIdx.x;
  const int64_t ch = chain_of(c.chain_mat_off, c.n_chains, m);
  const double F = c.F[ch], r = c.r[ch], T = c.T[m];
  const double D = exp(-r * T), sqT = sqrt(T);
  double th[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) th[j] = theta[m * 5 + j];
  const double inv_n = 1.0 / (double)c.n;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = c.mat_quote_off[m] + threadIdx.x; i < c.mat_quote_off[m + 1];
       i += blockDim.x) {
    const double K = c.K[i];
    const int fl = c.flag[i];
    const SviPoint sp = svi_eval(th, log(K / F));
    if (!(sp.w > kWMin)) continue;
    const double sigma = sqrt(sp.w / T);
    const double tgt = c.iv_target[i];
    if (!fv::finite_d(tgt)) continue;
    const double P = fv::price_at(F, K, D, sigma, sqT, fl);
    const fv::Reduced rd = fv::reduce_quote(fv::kBlack76, P, F, K, T, r, 0.0, fl);
    // IV(P(sigma)) through the LBR solver; where the model price is not
    // solvable in binary64 (it rounded onto the intrinsic value or the upper
    // bound) the composite takes its exact value sigma and unit slope
    double iv = sigma, ratio = 1.0;
    if (rd.status == fv::kQOk) {
      const fv::LbrResult res = fv::lbr_solve(rd.x, rd.beta, rd.bmax, 2, 4, 1e-6);
      iv = res.s / sqT;
      // vega(v) = D F phi(d1(v)) sqrt(T); only vega(sigma)/vega(iv) enters
      const double lfk = log(F / K);
      const double s1 = sigma * sqT, s2 = iv * sqT;
      const double d1a = lfk / s1 + 0.5 * s1, d1b = lfk / s2 + 0.5 * s2;
      ratio = exp(-0.5 * (d1a * d1a - d1b * d1b));
    }
    const double e = iv - tgt;
    const double g_sigma = 2.0 * e * inv_n * ratio;
    const double g_w = g_sigma / (2.0 * sigma * T);
    acc[0] += g_w * sp.dw[0];
    acc[1] += g_w * sp.dw[1];
    acc[2] += g_w * sp.dw[2];
    acc[3] += g_w * sp.dw[3];
    acc[4] += g_w * sp.dw[4];
    acc[5] += e * e;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int w = kCalibBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < 6; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < 5; ++j) grad[m * 5 + j] = red[j][0];
    loss_parts[m] = red[5][0];
  }
}

__global__ void k_svi_adam(int64_t n_par, double* __restrict__ theta, double* __restrict__ am,
                           double* __restrict__ av, const double* __restrict__ grad,
                           const int64_t* __restrict__ step, double lr, double b1, double b2,
                           double eps) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_par) return;
  const double t = (double)(*step + 1);
  const double g = grad[j];
  const double m = b1 * am[j] + (1.0 - b1) * g;
  const double v = b2 * av[j] + (1.0 - b2) * g * g;
  am[j] = m;
  av[j] = v;
  const double mh = m / (1.0 - pow(b1, t));
  const double vh = v / (1.0 - pow(b2, t));
  theta[j] -= lr * mh / (sqrt(vh) + eps);
}

__global__ __launch_bounds__(kCalibBlock) void k_svi_finish(int64_t n_mat, int64_t n,
                                                            const double* __restrict__ parts,
                                                            double* __restrict__ loss,
                                                            int64_t loss_len,
                                                            int64_t* __restrict__ step) {
  __shared__ double red[kCalibBlock];
  double a = 0.0;
  for (int64_t m = threadIdx.x; m < n_mat; m += blockDim.x) a += parts[m];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = kCalibBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t t = *step;
    if (loss && t >= 0 && t < loss_len) loss[t] = red[0] / (double)n;
    *step = t + 1;
  }
}

__global__ void k_svi_vols(KSvi c, const double* __restrict__ theta, double* __restrict__ out) {
  const int64_t m = blockIdx.x;
  const double T = c.T[m];
  const int64_t ch = chain_of(c.chain_mat_off, c.n_chains, m);
  const double F = c.F[ch];
  double th[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) th[j] = theta[m * 5 + j];
  for (int64_t i = c.mat_quote_off[m] + threadIdx.x; i < c.mat_quote_off[m + 1];
       i += blockDim.x) {
    const SviPoint sp = svi_eval(th, log(c.K[i] / F));
    out[i] = sp.w > 0.0 ? sqrt(sp.w / T) : __builtin_nan("");
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
  k_svi_grad<<<dim3((unsigned)k.n_mat), dim3(kCalibBlock), 0, s>>>(k, theta, grad, loss_parts);
  const int64_t n_par = 5 * k.n_mat;
  k_svi_adam<<<dim3((unsigned)((n_par + 255) / 256)), dim3(256), 0, s>>>(
      n_par, theta, adam_m, adam_v, grad, step, p->lr, p->beta1, p->beta2, p->eps);
  k_svi_finish<<<dim3(1), dim3(kCalibBlock), 0, s>>>(k.n_mat, k.n, loss_parts, loss, loss_len,
                                                    step);
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
