/* fv_capi_demo.c -- a plain C caller of the library: no Python, no torch.
 *
 * Allocates device memory with the HIP runtime, draws a seeded batch of
 * Black-Scholes-Merton quotes on the host (S = 100, K = S e^u with
 * u ~ U[-1/2, 1/2], T ~ U[0.02, 2], r ~ U[0, 0.05], q ~ U[0, 0.03],
 * sigma ~ U[0.05, 1], calls and puts alternating), prices them with
 * fv_price, inverts the prices with fv_implied_vol (both solvers) and checks
 * the round trip sigma -> price -> sigma: every quote must come back with
 * status FV_Q_OK and within max(tol sigma, 64 u (P + D F + D K) / vega) of
 * its sigma -- the binary64 price carries rounding errors at the scale of the
 * discounted forward and strike, not of the price itself, and the inversion
 * turns a price error into a sigma error divided by vega (from fv_greeks);
 * tol is 1e-12 (LBR) or 1e-8 (Halley) relative.  Quotes whose price lies
 * within 64 ulps of its intrinsic value or of its upper bound may instead
 * carry a bound status (deep in the money, the time value lost to rounding:
 * the price no longer determines sigma).  Each call is then timed with HIP
 * events on a stream of its own.
 *
 * Usage: fv_capi_demo [n] [reps]   (defaults 4096 and 100)
 * Prints one JSON line; exit status 0 when every check passes, 1 when a
 * check fails, 2 on a HIP or library error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fastvol.h"

#define HIP_OK(call)                                                         \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));      \
      exit(2);                                                               \
    }                                                                        \
  } while (0)

#define FV_OK_(call)                                                         \
  do {                                                                       \
    int r_ = (call);                                                         \
    if (r_ != FV_OK) {                                                       \
      fprintf(stderr, "%s failed (%d): %s\n", #call, r_, fv_last_error());   \
      exit(2);                                                               \
    }                                                                        \
  } while (0)

/* xorshift64* -> uniform in [0, 1) */
static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double unif(void) {
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 0x2545F4914F6CDD1Dull) >> 11) * 0x1p-53;
}

static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

static double* dalloc(int64_t n) {
  void* p = NULL;
  HIP_OK(hipMalloc(&p, (size_t)(n > 0 ? n : 1) * sizeof(double)));
  return (double*)p;
}

int main(int argc, char** argv) {
  const int64_t n = argc > 1 ? atoll(argv[1]) : 4096;
  const int reps = argc > 2 ? atoi(argv[2]) : 100;
  if (n <= 0 || reps <= 0) {
    fprintf(stderr, "usage: fv_capi_demo [n > 0] [reps > 0]\n");
    return 2;
  }
  const double u = 0x1p-53;
  double* hS = malloc(n * sizeof(double));
  double* hK = malloc(n * sizeof(double));
  double* hT = malloc(n * sizeof(double));
  double* hr = malloc(n * sizeof(double));
  double* hq = malloc(n * sizeof(double));
  double* hsig = malloc(n * sizeof(double));
  double* hP = malloc(n * sizeof(double));
  double* hvega = malloc(n * sizeof(double));
  double* hback = malloc(n * sizeof(double));
  uint8_t* hst = malloc(n);
  int8_t* hfl = malloc(n);
  double* times = malloc(reps * sizeof(double));
  if (!hS || !hK || !hT || !hr || !hq || !hsig || !hP || !hvega || !hback || !hst || !hfl ||
      !times) {
    fprintf(stderr, "host allocation failed\n");
    return 2;
  }
  for (int64_t i = 0; i < n; ++i) {
    hS[i] = 100.0;
    hK[i] = 100.0 * exp(unif() - 0.5);
    hT[i] = 0.02 + 1.98 * unif();
    hr[i] = 0.05 * unif();
    hq[i] = 0.03 * unif();
    hsig[i] = 0.05 + 0.95 * unif();
    hfl[i] = (i & 1) ? -1 : 1;
  }
  double *S = dalloc(n), *K = dalloc(n), *T = dalloc(n), *r = dalloc(n), *q = dalloc(n),
         *sig = dalloc(n), *P = dalloc(n), *vega = dalloc(n), *back = dalloc(n);
  uint8_t* st = NULL;
  int8_t* fl = NULL;
  HIP_OK(hipMalloc((void**)&st, (size_t)n));
  HIP_OK(hipMalloc((void**)&fl, (size_t)n));
  HIP_OK(hipMemcpy(S, hS, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(K, hK, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(T, hT, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(r, hr, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(q, hq, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(sig, hsig, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(fl, hfl, (size_t)n, hipMemcpyHostToDevice));
  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));

  fv_quotes qs;
  qs.n = n;
  qs.price.ptr = P;   qs.price.value = 0.0;
  qs.fs.ptr = S;      qs.fs.value = 0.0;
  qs.K.ptr = K;       qs.K.value = 0.0;
  qs.T.ptr = T;       qs.T.value = 0.0;
  qs.r.ptr = r;       qs.r.value = 0.0;
  qs.q.ptr = q;       qs.q.value = 0.0;
  qs.flag = fl;
  qs.flag_value = 1;
  fv_arg sarg;
  sarg.ptr = sig;
  sarg.value = 0.0;

  FV_OK_(fv_price(FV_MODEL_BSM, &qs, sarg, P, s));
  FV_OK_(fv_greeks(FV_MODEL_BSM, &qs, sarg, NULL, NULL, vega, NULL, NULL, s));
  HIP_OK(hipStreamSynchronize(s));
  HIP_OK(hipMemcpy(hP, P, n * sizeof(double), hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(hvega, vega, n * sizeof(double), hipMemcpyDeviceToHost));

  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  int failures = 0;
  printf("{\"n\": %lld, \"reps\": %d", (long long)n, reps);
  for (int solver = FV_SOLVER_LBR; solver <= FV_SOLVER_HALLEY; ++solver) {
    FV_OK_(fv_implied_vol(FV_MODEL_BSM, solver, &qs, back, st, NULL, s));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipMemcpy(hback, back, n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hst, st, (size_t)n, hipMemcpyDeviceToHost));
    const double tol = solver == FV_SOLVER_LBR ? 1e-12 : 1e-8;
    int64_t bad = 0, at = 0;
    double worst = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double F = hS[i] * exp((hr[i] - hq[i]) * hT[i]), D = exp(-hr[i] * hT[i]);
      const double I = D * fmax(hfl[i] * (F - hK[i]), 0.0);
      const double M = D * (hfl[i] > 0 ? F : hK[i]);
      const int boundary = fabs(hP[i] - I) <= 64.0 * u * fmax(hP[i], I) ||
                           fabs(M - hP[i]) <= 64.0 * u * M;
      if (boundary && hst[i] != FV_Q_OK) {
        ++at;
        continue;
      }
      const double lim = fmax(tol * hsig[i], 64.0 * u * (hP[i] + D * (F + hK[i])) / hvega[i]);
      const double err = fabs(hback[i] - hsig[i]);
      if (hst[i] != FV_Q_OK || !(err <= lim)) {
        ++bad;
      } else if (err / lim > worst) {
        worst = err / lim;
      }
    }
    for (int k = 0; k < 3; ++k) FV_OK_(fv_implied_vol(FV_MODEL_BSM, solver, &qs, back, st, NULL, s));
    for (int k = 0; k < reps; ++k) {
      HIP_OK(hipEventRecord(e0, s));
      FV_OK_(fv_implied_vol(FV_MODEL_BSM, solver, &qs, back, st, NULL, s));
      HIP_OK(hipEventRecord(e1, s));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      times[k] = ms;
    }
    qsort(times, reps, sizeof(double), cmp_double);
    const double med_ms = times[reps / 2];
    printf(", \"%s\": {\"bad\": %lld, \"at_bound\": %lld, \"worst_err_over_tol\": %.3g, "
           "\"median_us\": %.2f, \"implied_vols_per_s\": %.4g}",
           solver == FV_SOLVER_LBR ? "lbr" : "halley", (long long)bad, (long long)at, worst,
           med_ms * 1e3, (double)n / (med_ms * 1e-3));
    failures += bad > 0;
  }
  printf(", \"ok\": %s}\n", failures ? "false" : "true");
  HIP_OK(hipEventDestroy(e0));
  HIP_OK(hipEventDestroy(e1));
  HIP_OK(hipStreamDestroy(s));
  hipFree(S); hipFree(K); hipFree(T); hipFree(r); hipFree(q); hipFree(sig); hipFree(P);
  hipFree(vega); hipFree(back); hipFree(st); hipFree(fl);
  free(hS); free(hK); free(hT); free(hr); free(hq); free(hsig); free(hP); free(hvega);
  free(hback); free(hst); free(hfl); free(times);
  return failures ? 1 : 0;
}
