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
// One step = four launches, all graph-capturable (no allocation, no host
// synchronisation, no memset), with a workspace the caller provides:
//   1. per maturity: the natural parameters into a table (the
//      softplus/tanh transforms run once per maturity, not once per quote);
//   2. flat over the quotes, one wave per 64 consecutive quotes: SVI ->
//      Black-76 price -> LBR implied volatility -> residual -> adjoint
//      (dIV/dP = 1/vega(IV), dP/dsigma = vega(sigma), dsigma/dw =
//      1/(2 sigma T)), then a segmented sum over the wave's lanes keyed by
//      maturity; the head lane of every (wave, maturity) run stores the six
//      sums at index wave + maturity (unique: along the quotes both indices
//      only grow, and each run changes at least one), so no atomics are
//      needed and results are bitwise reproducible; its first thread also
//      advances the step counter and forms Adam's bias corrections;
//   3. one wave per maturity: the sums of its runs (lanes over runs, then a
//      fixed butterfly) -> gradient -> Adam update; each workgroup stores
//      the squared-error sum of its maturities;
//   4. one workgroup: the loss, a fixed-order sum of those.
// The price is handed to the solver in the normalised coordinates it
// reduces every quote to: the Black-76 price of the model is
// D sqrt(F K) (b(x, s) + intrinsic), and the solver's reduction (undiscount,
// subtract the intrinsic value, divide by sqrt(F K)) takes it back to
// beta = b(x, s) exactly in exact arithmetic, so the kernel passes beta = b
// of the out-of-the-money side to the LBR solve without the round trip.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>

#include "../../include/fastvol.h"
#include "fv_csr.h"
#include "fv_host.h"
#include "fv_quote.h"

namespace {

constexpr int kCalibBlock = 256;
constexpr double kWMin = 1e-10;  // total variance floor: quotes below it are skipped

// Per-maturity record of the natural parameters (k_svi_prep), read by
// k_svi_grad and k_svi_adam.
enum NatField : int {
  kNatA, kNatMu, kNatT,
  kNatB, kNatRho, kNatS,
  kNatSigB,   // softplus'(b~) = sigmoid(b~)
  kNatSigS,   // softplus'(s~) = sigmoid(s~)
  kNatCount
};
// Per (wave, maturity) run: the six sums of the adjoint.
enum SumField : int {
  kSumG,       // sum g_w,               g_w = dL/dw of a quote
  kSumGRt,     // sum g_w sqrt((k - m)^2 + s^2)
  kSumGDk,     // sum g_w (k - m)
  kSumGDkIrt,  // sum g_w (k - m) / sqrt((k - m)^2 + s^2)
  kSumGIrt,    // sum g_w / sqrt((k - m)^2 + s^2)
  kSumE2,      // sum (IV - target)^2
  kSumCount
};
// Control block at the start of the workspace: Adam's bias corrections of
// the step.
enum CtlField : int { kCtlC1, kCtlC2, kCtlCount };

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

constexpr int kWavesPerBlock = kCalibBlock / 64;
int64_t n_waves_of(int64_t n) { return (n + 63) / 64; }
int64_t n_adam_blocks(int64_t n_mat) { return (n_mat + kWavesPerBlock - 1) / kWavesPerBlock; }

// workspace layout (doubles): control block, per-maturity records, per
// workgroup squared-error sums of k_svi_adam, then the run sums
int64_t workspace_doubles(int64_t n_mat, int64_t n) {
  return kCtlCount + kNatCount * n_mat + n_adam_blocks(n_mat) +
         kSumCount * (n_waves_of(n) + n_mat);
}

struct Workspace {
  double* ctl;
  double* nat;
  double* block_e2;
  double* part;
};

Workspace carve(double* ws, int64_t n_mat) {
  Workspace w;
  w.ctl = ws;
  w.nat = ws + kCtlCount;
  w.block_e2 = w.nat + kNatCount * n_mat;
  w.part = w.block_e2 + n_adam_blocks(n_mat);
  return w;
}

// Natural parameters of one maturity from its raw parameters.
struct SviMat {
  double a, b, rho, mu, s, T;
};

__device__ __forceinline__ SviMat svi_mat(const double* __restrict__ theta,
                                          const double* __restrict__ T, int64_t m) {
  const double* th = theta + 5 * m;
  SviMat q;
  q.a = th[0];
  q.b = softplus(th[1]);
  q.rho = tanh(th[2]);
  q.mu = th[3];
  q.s = softplus(th[4]);
  q.T = T[m];
  return q;
}

// sqrt((k - m)^2 + s^2) and its reciprocal: the refined hardware reciprocal
// square root where the radicand is a normal number, the library square
// root otherwise (s underflowed to 0 at k = m)
__device__ __forceinline__ void svi_root(double u, double& rt, double& irt) {
  if (u >= 2.2250738585072014e-308) {
    irt = fv::rsqrt(u);
    rt = u * irt;
  } else {
    rt = sqrt(u);
    irt = 1.0 / rt;
  }
}

__global__ __launch_bounds__(kCalibBlock) void k_svi_prep(int64_t n_mat,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ theta,
                                                          double* __restrict__ nat) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_mat) return;
  const SviMat q = svi_mat(theta, T, m);
  double* o = nat + kNatCount * m;
  o[kNatA] = q.a;
  o[kNatMu] = q.mu;
  o[kNatT] = q.T;
  o[kNatB] = q.b;
  o[kNatRho] = q.rho;
  o[kNatS] = q.s;
  o[kNatSigB] = sigmoid(theta[5 * m + 1]);
  o[kNatSigS] = sigmoid(theta[5 * m + 4]);
}

__global__ __launch_bounds__(kCalibBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_svi_grad(
    KSvi c, const double* __restrict__ nat, double* __restrict__ ctl, double* __restrict__ part,
    int64_t* __restrict__ step, double b1, double b2) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the step's counter and bias corrections; nothing else in this launch
    // reads them, k_svi_adam runs after it on the stream
    const int64_t t = *step + 1;
    *step = t;
    ctl[kCtlC1] = 1.0 - pow(b1, (double)t);
    ctl[kCtlC2] = 1.0 - pow(b2, (double)t);
  }
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = (int)__lane_id();
  const int64_t w0 = wave * 64;
  if (w0 >= c.n) return;  // wave-uniform
  fv::ChainCursor cur;
  cur.init(c.mat_quote_off, c.n_mat, c.chain_mat_off, c.n_chains, w0);
  const int64_t i = w0 + lane;
  int64_t m, cc;
  cur.slice(w0, min(w0 + 63, c.n - 1), i, m, cc);
  SviMat q;
  {
    const double* r = nat + kNatCount * m;
    q.a = r[kNatA];
    q.b = r[kNatB];
    q.rho = r[kNatRho];
    q.mu = r[kNatMu];
    q.s = r[kNatS];
    q.T = r[kNatT];
  }
  double v[kSumCount];
#pragma unroll
  for (int j = 0; j < kSumCount; ++j) v[j] = 0.0;
  if (i < c.n) {
    const double tgt = c.iv_target[i];
    const double fk = c.F[cc] * fv::rcp(c.K[i]);
    const double lfk = fv::flog(fk);  // ln(F/K) = -k
    const double dk = -lfk - q.mu;
    double rt, irt;
    svi_root(fma(dk, dk, q.s * q.s), rt, irt);
    const double w = fma(q.b, fma(q.rho, dk, rt), q.a);
    if (w > kWMin && fv::finite_d(tgt)) {
      const double iT = fv::rcp(q.T);
      const double vv = w * iT;
      const double sigma = vv * fv::rsqrt(vv);
      const double isqT = fv::rsqrt(q.T);
      const double s1 = sigma * (q.T * isqT);
      // out-of-the-money side: x = -|ln(F/K)| <= 0, beta = b(x, s1),
      // b_max = e^{x/2} = sqrt(min(F/K, K/F))
      const double x = -fabs(lfk);
      const double bmax = fk < 1.0 ? fk * fv::rsqrt(fk) : fv::rsqrt(fk);
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
        // vega(v) = D F phi(d1(v)) sqrt(T); only vega(sigma)/vega(iv) enters:
        // with s = v sqrt(T) and d1 = ln(F/K)/s + s/2,
        //   ln(vega(s1)/vega(s2)) = -(d1(s1)^2 - d1(s2)^2)/2
        //                         = -(s1^2 - s2^2)(1/4 - L^2)/2,  L = ln(F/K)/(s1 s2),
        // which vanishes up to rounding (IV(P(sigma)) = sigma)
        const double s2 = res.s;
        const double L = lfk * fv::rcp(s1 * s2);
        const double dl = -0.5 * (s1 - s2) * (s1 + s2) * fma(-L, L, 0.25);
        ratio = fabs(dl) < 1e-8 ? 1.0 + dl : fv::fexp(dl);
      }
      const double e = iv - tgt;
      // dL/dw = (2 e/N) ratio / (2 sigma T), with 1/N applied per maturity sum
      const double g_w = e * ratio * fv::rcp(sigma * q.T);
      v[kSumG] = g_w;
      v[kSumGRt] = g_w * rt;
      v[kSumGDk] = g_w * dk;
      v[kSumGDkIrt] = g_w * dk * irt;
      v[kSumGIrt] = g_w * irt;
      v[kSumE2] = e * e;
    }
  }
  // Segmented suffix sums over the lanes keyed by maturity: the maturity is
  // non-decreasing along the lanes, so equal keys at distance `off` enclose
  // a run of equal keys and each lane ends with the sum from itself to the
  // end of its run.  Lanes past the last quote carry zeros and the last
  // quote's maturity.
  const int key = (int)(m - fv::readlane64(m, 0));
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int nk = __shfl_down(key, off);
    const bool add = lane + off < 64 && nk == key;
#pragma unroll
    for (int j = 0; j < kSumCount; ++j) {
      const double o = __shfl_down(v[j], off);
      if (add) v[j] += o;
    }
  }
  const int pk = __shfl_up(key, 1);
  if ((lane == 0 || pk != key) && i < c.n) {
    double* o = part + kSumCount * (wave + m);
#pragma unroll
    for (int j = 0; j < kSumCount; ++j) o[j] = v[j];
  }
}

// loss[t - 1] = (1/N) sum of k_svi_adam's per-workgroup squared-error sums,
// in a fixed order (one workgroup: strided partial sums, then a tree).
constexpr int kLossBlock = 1024;
__global__ __launch_bounds__(kLossBlock) void k_svi_loss(int64_t nb, int64_t n,
                                                         const double* __restrict__ block_e2,
                                                         const int64_t* __restrict__ step,
                                                         double* __restrict__ loss,
                                                         int64_t loss_len) {
  __shared__ double red[kLossBlock];
  double a = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kLossBlock) a += block_e2[b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int wd = kLossBlock / 2; wd > 0; wd >>= 1) {
    if ((int)threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
    __syncthreads();
  }
  const int64_t t = *step;
  if (threadIdx.x == 0 && t >= 1 && t <= loss_len) loss[t - 1] = red[0] * (1.0 / (double)n);
}

// Adam with the counter and bias corrections k_svi_grad set, one wave per
// maturity: lane l sums the maturity's runs l, l + 64, ... in order, a fixed
// butterfly over the lanes completes the six sums (every lane ends with the
// same totals), and lane j < 5 updates parameter j.  Each workgroup stores
// the squared-error sum of its maturities, in wave order, for k_svi_loss.
__global__ __launch_bounds__(kCalibBlock) void k_svi_adam(
    int64_t n_mat, int64_t n, const int64_t* __restrict__ mat_quote_off,
    const double* __restrict__ nat, const double* __restrict__ part, double* __restrict__ theta,
    double* __restrict__ am, double* __restrict__ av, double* __restrict__ grad,
    const double* __restrict__ ctl, double* __restrict__ block_e2, double lr, double b1,
    double b2, double eps) {
  __shared__ double wave_e2[kWavesPerBlock];
  const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = (int)__lane_id();
  const int wib = (int)(threadIdx.x >> 6);
  double S[kSumCount];
#pragma unroll
  for (int j = 0; j < kSumCount; ++j) S[j] = 0.0;
  bool empty = true;
  if (m < n_mat) {  // wave-uniform
    const int64_t q0 = mat_quote_off[m], q1 = mat_quote_off[m + 1];
    empty = q1 <= q0;  // an empty maturity has no runs and no record
    if (!empty) {
      for (int64_t w = (q0 >> 6) + lane; w <= (q1 - 1) >> 6; w += 64) {
        const double* o = part + kSumCount * (w + m);
#pragma unroll
        for (int j = 0; j < kSumCount; ++j) S[j] += o[j];
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int j = 0; j < kSumCount; ++j) S[j] += __shfl_xor(S[j], off);
    }
    if (lane < 5) {
      double g = 0.0;
      if (!empty) {
        const double* q = nat + kNatCount * m;
        const double b = q[kNatB], rho = q[kNatRho];
        // dL/dtheta = (1/N) sum g_w dw/dtheta with
        //   dw/da = 1, dw/db~ = (rho dk + rt) sigmoid(b~), dw/drho~ = b dk (1 - rho^2),
        //   dw/dm = -b (rho + dk/rt), dw/ds~ = b (s/rt) sigmoid(s~)
        switch (lane) {
          case 0: g = S[kSumG]; break;
          case 1: g = fma(rho, S[kSumGDk], S[kSumGRt]) * q[kNatSigB]; break;
          case 2: g = b * (1.0 - rho * rho) * S[kSumGDk]; break;
          case 3: g = -b * fma(rho, S[kSumG], S[kSumGDkIrt]); break;
          default: g = b * q[kNatS] * q[kNatSigS] * S[kSumGIrt]; break;
        }
        g *= 1.0 / (double)n;
      }
      const int64_t k = 5 * m + lane;
      grad[k] = g;
      const double mo = b1 * am[k] + (1.0 - b1) * g;
      const double vo = b2 * av[k] + (1.0 - b2) * g * g;
      am[k] = mo;
      av[k] = vo;
      theta[k] -= lr * (mo / ctl[kCtlC1]) / (sqrt(vo / ctl[kCtlC2]) + eps);
    }
  }
  if (lane == 0) wave_e2[wib] = S[kSumE2];
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int j = 0; j < kWavesPerBlock; ++j) a += wave_e2[j];
    block_e2[blockIdx.x] = a;
  }
}

__global__ void k_svi_vols(KSvi c, const double* __restrict__ theta, double* __restrict__ out) {
  const int64_t m = blockIdx.x;
  const double T = c.T[m];
  int64_t lo = 0, hi = c.n_chains;  // chain of maturity m: largest lo with off[lo] <= m
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (c.chain_mat_off[mid] <= m) lo = mid; else hi = mid;
  }
  const double F = c.F[lo];
  const double* th = theta + 5 * m;
  const double a = th[0], b = softplus(th[1]), rho = tanh(th[2]), mu = th[3], s = softplus(th[4]);
  for (int64_t i = c.mat_quote_off[m] + threadIdx.x; i < c.mat_quote_off[m + 1];
       i += blockDim.x) {
    const double dk = log(c.K[i] / F) - mu;
    const double w = a + b * (rho * dk + sqrt(dk * dk + s * s));
    out[i] = w > 0.0 ? sqrt(w / T) : __builtin_nan("");
  }
}

int check_problem(const fv_svi_problem* p) {
  if (!p) return fvh::fail(FV_E_INVALID_ARG, "problem pointer is NULL");
  const fv_chains& c = p->chains;
  if (c.n_chains <= 0 || c.n_maturities <= 0 || c.n_quotes <= 0)
    return fvh::fail(FV_E_INVALID_ARG, "empty or negative chain sizes");
  if (c.n_maturities > 0x7fffffff || c.n_quotes > ((int64_t)1 << 46))
    return fvh::fail(FV_E_INVALID_ARG, "too many maturities or quotes");
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

// The four launches of one step, with the workspace `ws` (at least
// workspace_doubles(n_mat, n) doubles, checked by the callers).
int launch_step(const fv_svi_problem* p, double* theta, double* adam_m, double* adam_v,
                int64_t* step, double* grad, double* ws, double* loss, int64_t loss_len,
                void* stream) {
  if (!p->iv_target || !theta || !adam_m || !adam_v || !step || !grad)
    return fvh::fail(FV_E_INVALID_ARG, "NULL parameter, state or gradient array");
  if (loss_len < 0) return fvh::fail(FV_E_INVALID_ARG, "loss_len < 0");
  if (!(p->lr > 0.0) || !(p->beta1 >= 0.0 && p->beta1 < 1.0) ||
      !(p->beta2 >= 0.0 && p->beta2 < 1.0) || !(p->eps > 0.0))
    return fvh::fail(FV_E_INVALID_ARG, "Adam hyper-parameters out of range");
  const KSvi k = to_k(p);
  hipStream_t s = (hipStream_t)stream;
  const Workspace w = carve(ws, k.n_mat);
  const int64_t waves = n_waves_of(k.n);
  const int64_t nb = n_adam_blocks(k.n_mat);
  k_svi_prep<<<dim3((unsigned)((k.n_mat + kCalibBlock - 1) / kCalibBlock)), dim3(kCalibBlock), 0,
               s>>>(k.n_mat, k.T, theta, w.nat);
  k_svi_grad<<<dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)), dim3(kCalibBlock),
               0, s>>>(k, w.nat, w.ctl, w.part, step, p->beta1, p->beta2);
  k_svi_adam<<<dim3((unsigned)nb), dim3(kCalibBlock), 0, s>>>(
      k.n_mat, k.n, k.mat_quote_off, w.nat, w.part, theta, adam_m, adam_v, grad, w.ctl,
      w.block_e2, p->lr, p->beta1, p->beta2, p->eps);
  if (loss && loss_len > 0)
    k_svi_loss<<<dim3(1), dim3(kLossBlock), 0, s>>>(nb, k.n, w.block_e2, step, loss, loss_len);
  return fvh::launched("fv_svi_adam_step");
}

// Workspace of the allocation-free step: one array per GPU, part of the
// library's code object (each device that loads the library holds its own
// copy until the process ends).  Host code never passes `scratch` itself to
// a kernel (on the host the name is only a stand-in): it takes the device
// address from hipGetSymbolAddress, once per device, with that device
// current.
constexpr int64_t kScratchDoubles = (int64_t)1 << 20;  // 8 MiB
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::atomic<double*> g_scratch_ptr[kMaxDevices];

// Device address of the current device's `scratch` into *out; FV_OK or an
// FV_E_* code with its text set.
int scratch_of_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fvh::fail(FV_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fvh::fail(FV_E_UNSUPPORTED, "device ordinal beyond the 64 the library tracks");
  double* ptr = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (!ptr) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ptr = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!ptr) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fvh::fail(FV_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       (e != hipSuccess ? hipGetErrorString(e) : "NULL address"));
      ptr = static_cast<double*>(p);
      g_scratch_ptr[dev].store(ptr, std::memory_order_release);
    }
  }
  *out = ptr;
  return FV_OK;
}

}  // namespace

extern "C" {

int64_t fv_svi_workspace_size(const fv_svi_problem* p) {
  const int rc = check_problem(p);
  if (rc) return rc;
  return workspace_doubles(p->chains.n_maturities, p->chains.n_quotes);
}

int fv_svi_adam_step(const fv_svi_problem* p, double* theta, double* adam_m, double* adam_v,
                     int64_t* step, double* grad, double* workspace, int64_t workspace_len,
                     double* loss, int64_t loss_len, void* stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  if (!workspace) return fvh::fail(FV_E_INVALID_ARG, "workspace is NULL");
  if (workspace_len < workspace_doubles(p->chains.n_maturities, p->chains.n_quotes))
    return fvh::fail(FV_E_INVALID_ARG, "workspace smaller than fv_svi_workspace_size()");
  return launch_step(p, theta, adam_m, adam_v, step, grad, workspace, loss, loss_len, stream);
}

int fv_svi_adam_step_noalloc(const fv_svi_problem* p, double* theta, double* adam_m,
                             double* adam_v, int64_t* step, double* grad, double* loss,
                             int64_t loss_len, void* stream) {
  int rc = check_problem(p);
  if (rc) return rc;
  const int64_t need = workspace_doubles(p->chains.n_maturities, p->chains.n_quotes);
  if (need > kScratchDoubles)
    return fvh::fail(FV_E_INVALID_ARG,
                     "problem needs " + std::to_string(need) +
                         " doubles of workspace; the allocation-free step holds at most " +
                         std::to_string(kScratchDoubles) + " (8 MiB): use fv_svi_adam_step");
  double* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  return launch_step(p, theta, adam_m, adam_v, step, grad, ws, loss, loss_len, stream);
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
