// fv_kernels.hip -- gfx950 kernels and the C ABI declared in include/fastvol.h.
//
// Every kernel is a single pass over struct-of-arrays FP64 inputs: each lane
// loads its quote once (coalesced: consecutive lanes read consecutive
// quotes), keeps the whole solve in registers and stores once.  A thread
// handles `qpt` quotes spaced one block apart so that every load of a wave
// stays one contiguous 512-byte segment.  Divergent regions (solver
// branches, extra Householder steps, rare evaluator forms) are plain
// per-lane control flow: the hardware skips a side whose exec mask is empty,
// so a wave pays only for the branches its own lanes take.  The Halley
// kernel compacts its non-converged lanes with wave ballots into an LDS
// queue and runs the bisection fallback over the packed queue.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <string>
#include <vector>

#include "../../include/fastvol.h"
#include "fv_f32.h"
#include "fv_host.h"
#include "fv_csr.h"
#include "fv_quote.h"

// Error state shared by every entry point of the library (fv_host.h).
namespace fvh {
thread_local std::string g_last_error;
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
int launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FV_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return FV_OK;
}
}  // namespace fvh

namespace {

using fv::Greeks;
using fv::IvGrad;
using fv::LbrResult;
using fv::Reduced;

// ------------------------------------------------------------- arguments
struct KQuotes {
  int64_t n;
  fv_arg price, fs, K, T, r, q;
  const int8_t* flag;
  int8_t flag_value;
  int hsteps;  // Halley steps before the bisection fallback (fv_set_halley_steps)
};

// A field's value for quote i: its array entry, or its broadcast value.
// ARR = true is the specialisation for calls whose per-quote fields are all
// arrays (checked on the host): the pointer-or-value choice per field and
// its condition, which the solver kernels otherwise keep across the whole
// solve, disappear.
template <bool ARR = false>
__device__ __forceinline__ double ld(const fv_arg& a, int64_t i) {
  return ARR ? a.ptr[i] : (a.ptr ? a.ptr[i] : a.value);
}
template <bool ARR = false>
__device__ __forceinline__ int ldflag(const KQuotes& q, int64_t i) {
  return ARR ? (int)q.flag[i] : (q.flag ? (int)q.flag[i] : (int)q.flag_value);
}

struct GreekOut {
  double* p[5];
  int any;
};

// LBR iteration policy: two Householder(3) steps always; a third (and at most
// a fourth) only while the previous step still moved s by more than 1e-6
// relative, i.e. only in waves that hold such a lane.
// Largest workgroup the kernels are compiled for (8 waves).
constexpr int kMaxBlock = 512;
// Minimum resident waves per SIMD the solver kernels are register-allocated
// for (2: up to 256 VGPRs, 3: 168, 4: 128, 6: 80).  LBR runs at 4: at 6 it
// is no faster, and its one-byte flag and status accesses (half a 128-byte
// line per wave) then get fetched and written back twice as often (53 + 13
// instead of 49 + 9 bytes per quote on the wide workload).  The Halley
// kernels, at 80 VGPRs without spills, run 6.  The fused-Greeks variants
// keep more live values and are held at 2 so that they do not spill.
#ifndef FV_LBR_WAVES_PER_EU
#define FV_LBR_WAVES_PER_EU 4
#endif
#ifndef FV_HALLEY_WAVES_PER_EU
#define FV_HALLEY_WAVES_PER_EU 6
#endif
#define FV_WAVES_LBR(GREEKS) ((GREEKS) ? 2 : FV_LBR_WAVES_PER_EU)
#define FV_WAVES_HALLEY(GREEKS) ((GREEKS) ? 2 : FV_HALLEY_WAVES_PER_EU)
// The ragged kernel: at least 6 waves per SIMD (<= 80 VGPRs); its LBR form
// takes 62 VGPRs, and its Halley form, which took 83 at a floor of 4, is
// 2.7% faster held to 80.
#ifndef FV_CHAINS_WAVES_PER_EU
#define FV_CHAINS_WAVES_PER_EU 6
#endif

constexpr int kLbrMinSteps = 2;
constexpr int kLbrMaxSteps = 4;
constexpr double kLbrStepTol = 1e-6;
constexpr int kHalleySteps = 8;  // the paper's count; the default of fv_set_halley_steps
constexpr int kMaxHalleySteps = 64;
constexpr double kBisectTol = 1e-13;

// ------------------------------------------------------------- price
template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_price(KQuotes q, fv_arg sigma, double* __restrict__ out, int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i), r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const double sg = ld(sigma, i);
    const int th = ldflag(q, i);
    double p = __builtin_nan("");
    if (fv::finite_d(fs) && fv::finite_d(K) && fv::finite_d(T) && fv::finite_d(r) &&
        fv::finite_d(qy) && fv::finite_d(sg) && fs > 0.0 && K > 0.0 && T > 0.0 &&
        sg >= 0.0 && (th == 1 || th == -1)) {
      const double F = fv::forward_of(MODEL, fs, T, r, qy);
      const double D = fv::fexp_prod(-r, T);
      p = fv::price_at(F, K, D, sg, fv::sqrt_pos(T), th);
    }
    out[i] = p;
  }
}

// ------------------------------------------------------------- IV: LBR
template <int MODEL, bool GREEKS, bool ARR>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(FV_WAVES_LBR(GREEKS)))) void k_iv_lbr(KQuotes q, double* __restrict__ sig_out, uint8_t* __restrict__ st_out,
                         GreekOut g, int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double P = ld<ARR>(q.price, i), fs = ld<ARR>(q.fs, i), K = ld<ARR>(q.K, i), T = ld<ARR>(q.T, i),
                 r = ld<ARR>(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld<ARR>(q.q, i) : 0.0;
    const int th = ldflag<ARR>(q, i);
    const Reduced rd = fv::reduce_quote(MODEL, P, fs, K, T, r, qy, th);
    uint8_t st = rd.status;
    double sg = st == fv::kQAtIntrinsic ? 0.0 : __builtin_nan("");
    if (st == fv::kQOk) {
      const LbrResult res = fv::lbr_solve(rd.x, rd.beta, rd.bmax, rd.lnb, kLbrMinSteps, kLbrMaxSteps, kLbrStepTol);
      sg = res.s * rd.isqrtT;
      if (!res.converged) st = fv::kQNotConverged;
    }
    sig_out[i] = sg;
    if (st_out) st_out[i] = st;
    if (GREEKS) {
      Greeks gr;
      if (st == fv::kQOk) {
        gr = fv::greeks_at(MODEL, fs, K, T, r, qy, sg, th, rd.F, rd.D, P);
      } else {
        const double nan = __builtin_nan("");
        gr.delta = gr.gamma = gr.vega = gr.theta = gr.rho = nan;
      }
      if (g.p[0]) g.p[0][i] = gr.delta;
      if (g.p[1]) g.p[1][i] = gr.gamma;
      if (g.p[2]) g.p[2][i] = gr.vega;
      if (g.p[3]) g.p[3][i] = gr.theta;
      if (g.p[4]) g.p[4][i] = gr.rho;
    }
  }
}

// Diagnostic twin of k_iv_lbr: the same per-quote solve, recording the path
// each quote takes (guess region, evaluation forms, number of steps).
template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_lbr_trace(KQuotes q, uint32_t* __restrict__ out,
                                                         int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double P = ld(q.price, i), fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i),
                 r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const Reduced rd = fv::reduce_quote(MODEL, P, fs, K, T, r, qy, ldflag(q, i));
    uint32_t code = 0xFFFFFFFFu;  // not solved (status != OK)
    if (rd.status == fv::kQOk) {
      code = 0;
      fv::lbr_solve(rd.x, rd.beta, rd.bmax, rd.lnb, kLbrMinSteps, kLbrMaxSteps, kLbrStepTol, &code);
    }
    out[i] = code;
  }
}

// Diagnostic twin of k_iv_halley: the number of Halley steps each quote
// takes, with bit 8 set when it fails the convergence check (and would go
// through the bisection fallback).
template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_halley_trace(KQuotes q, uint32_t* __restrict__ out,
                                                            int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double P = ld(q.price, i), fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i),
                 r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const Reduced rd = fv::reduce_quote(MODEL, P, fs, K, T, r, qy, ldflag(q, i));
    uint32_t code = 0xFFFFFFFFu;  // not solved (status != OK)
    if (rd.status == fv::kQOk) {
      const fv::HalleyState hs = fv::halley_solve(rd.x, rd.beta, rd.bmax, rd.lnb, q.hsteps);
      code = (uint32_t)hs.steps | (hs.converged ? 0u : 0x100u);
    }
    out[i] = code;
  }
}

// ------------------------------------------------------------- IV: Halley
// LDS queue entry of a lane that failed the convergence check.
struct Pending {
  int64_t i;
  double lo, hi;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

template <int MODEL, bool GREEKS, bool ARR>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(FV_WAVES_HALLEY(GREEKS)))) void k_iv_halley(KQuotes q, double* __restrict__ sig_out,
                            uint8_t* __restrict__ st_out, GreekOut g, int qpt) {
  extern __shared__ unsigned char smem_raw[];
  Pending* queue = reinterpret_cast<Pending*>(smem_raw);
  __shared__ int qcount;
  if (threadIdx.x == 0) qcount = 0;
  __syncthreads();

  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    bool fail = false;
    fv::HalleyState hs;
    hs.lo = 0.0;
    hs.hi = 0.0;
    if (i < q.n) {
      const double P = ld<ARR>(q.price, i), fs = ld<ARR>(q.fs, i), K = ld<ARR>(q.K, i), T = ld<ARR>(q.T, i),
                   r = ld<ARR>(q.r, i);
      const double qy = MODEL == fv::kBlackScholesMerton ? ld<ARR>(q.q, i) : 0.0;
      const int th = ldflag<ARR>(q, i);
      const Reduced rd = fv::reduce_quote(MODEL, P, fs, K, T, r, qy, th);
      uint8_t st = rd.status;
      double sg = st == fv::kQAtIntrinsic ? 0.0 : __builtin_nan("");
      if (st == fv::kQOk) {
        hs = fv::halley_solve(rd.x, rd.beta, rd.bmax, rd.lnb, q.hsteps);
        sg = hs.s * rd.isqrtT;
        fail = !hs.converged;
      }
      if (!fail) {
        sig_out[i] = sg;
        if (st_out) st_out[i] = st;
        if (GREEKS) {
          Greeks gr;
          if (st == fv::kQOk) {
            gr = fv::greeks_at(MODEL, fs, K, T, r, qy, sg, th, rd.F, rd.D, P);
          } else {
            const double nan = __builtin_nan("");
            gr.delta = gr.gamma = gr.vega = gr.theta = gr.rho = nan;
          }
          if (g.p[0]) g.p[0][i] = gr.delta;
          if (g.p[1]) g.p[1][i] = gr.gamma;
          if (g.p[2]) g.p[2][i] = gr.vega;
          if (g.p[3]) g.p[3][i] = gr.theta;
          if (g.p[4]) g.p[4][i] = gr.rho;
        }
      }
    }
    // wave-level compaction of the failing lanes into the LDS queue
    const uint64_t mask = __ballot(fail);
    if (mask) {
      int wbase = 0;
      const int cnt = __popcll(mask);
      const unsigned first = __ffsll((unsigned long long)mask) - 1;
      if (__lane_id() == first) wbase = atomicAdd(&qcount, cnt);
      wbase = __shfl(wbase, first);
      if (fail) {
        const int slot = wbase + __popcll(mask & lanemask_lt());
        queue[slot].i = i;
        queue[slot].lo = hs.lo;
        queue[slot].hi = hs.hi;
      }
    }
  }
  __syncthreads();
  // bisection fallback over the packed queue: every lane of a wave works
  const int m = qcount;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int64_t i = queue[j].i;
    const double P = ld<ARR>(q.price, i), fs = ld<ARR>(q.fs, i), K = ld<ARR>(q.K, i), T = ld<ARR>(q.T, i),
                 r = ld<ARR>(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld<ARR>(q.q, i) : 0.0;
    const int th = ldflag<ARR>(q, i);
    const Reduced rd = fv::reduce_quote(MODEL, P, fs, K, T, r, qy, th);
    const double s =
        fv::bisection_solve(rd.x, rd.beta, rd.bmax, rd.lnb, queue[j].lo, queue[j].hi, kBisectTol);
    const double sg = s * rd.isqrtT;
    sig_out[i] = sg;
    if (st_out) st_out[i] = fv::kQOk;
    if (GREEKS) {
      const Greeks gr = fv::greeks_at(MODEL, fs, K, T, r, qy, sg, th, rd.F, rd.D, P);
      if (g.p[0]) g.p[0][i] = gr.delta;
      if (g.p[1]) g.p[1][i] = gr.gamma;
      if (g.p[2]) g.p[2][i] = gr.vega;
      if (g.p[3]) g.p[3][i] = gr.theta;
      if (g.p[4]) g.p[4][i] = gr.rho;
    }
  }
}

// ------------------------------------------------------------- Greeks
// ------------------------------------------------------------- IV: Halley, binary32
struct KQuotes32 {
  int64_t n;
  fv_arg_f32 price, fs, K, T, r, q;
  const int8_t* flag;
  int8_t flag_value;
  int hsteps;
};

__device__ __forceinline__ float ld32(const fv_arg_f32& a, int64_t i) {
  return a.ptr ? a.ptr[i] : a.value;
}

struct Pending32 {
  int64_t i;
  float lo, hi;
};

// The binary32 twin of k_iv_halley: same per-lane Halley, same ballot + LDS
// compaction of the lanes that fail the convergence check and bisection over
// the packed queue, in float arithmetic throughout.
template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_iv_halley32(
    KQuotes32 q, float* __restrict__ sig_out, uint8_t* __restrict__ st_out, int qpt) {
  extern __shared__ unsigned char smem_raw[];
  Pending32* queue = reinterpret_cast<Pending32*>(smem_raw);
  __shared__ int qcount;
  if (threadIdx.x == 0) qcount = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    bool fail = false;
    fv32::HalleyState hs;
    hs.lo = 0.0f;
    hs.hi = 0.0f;
    if (i < q.n) {
      const float P = ld32(q.price, i), fs = ld32(q.fs, i), K = ld32(q.K, i),
                  T = ld32(q.T, i), r = ld32(q.r, i);
      const float qy = MODEL == fv::kBlackScholesMerton ? ld32(q.q, i) : 0.0f;
      const int th = q.flag ? (int)q.flag[i] : (int)q.flag_value;
      const fv32::Reduced rd = fv32::reduce_quote(MODEL, P, fs, K, T, r, qy, th);
      const uint8_t st = rd.status;
      float sg = st == fv::kQAtIntrinsic ? 0.0f : __builtin_nanf("");
      if (st == fv::kQOk) {
        hs = fv32::halley_solve(rd.x, rd.beta, rd.bmax, rd.lnb, q.hsteps);
        sg = hs.s / rd.sqrtT;
        fail = !hs.converged;
      }
      if (!fail) {
        sig_out[i] = sg;
        if (st_out) st_out[i] = st;
      }
    }
    const uint64_t mask = __ballot(fail);
    if (mask) {
      int wbase = 0;
      const int cnt = __popcll(mask);
      const unsigned first = __ffsll((unsigned long long)mask) - 1;
      if (__lane_id() == first) wbase = atomicAdd(&qcount, cnt);
      wbase = __shfl(wbase, first);
      if (fail) {
        const int slot = wbase + __popcll(mask & lanemask_lt());
        queue[slot].i = i;
        queue[slot].lo = hs.lo;
        queue[slot].hi = hs.hi;
      }
    }
  }
  __syncthreads();
  const int m = qcount;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int64_t i = queue[j].i;
    const float P = ld32(q.price, i), fs = ld32(q.fs, i), K = ld32(q.K, i), T = ld32(q.T, i),
                r = ld32(q.r, i);
    const float qy = MODEL == fv::kBlackScholesMerton ? ld32(q.q, i) : 0.0f;
    const int th = q.flag ? (int)q.flag[i] : (int)q.flag_value;
    const fv32::Reduced rd = fv32::reduce_quote(MODEL, P, fs, K, T, r, qy, th);
    const float s = fv32::bisection_solve(rd.x, rd.beta, rd.bmax, queue[j].lo, queue[j].hi, 2e-7f);
    sig_out[i] = s / rd.sqrtT;
    if (st_out) st_out[i] = fv::kQOk;
  }
}

template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_greeks(KQuotes q, fv_arg sigma, GreekOut g, int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i), r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const double sg = ld(sigma, i);
    const int th = ldflag(q, i);
    Greeks gr;
    const double nan = __builtin_nan("");
    gr.delta = gr.gamma = gr.vega = gr.theta = gr.rho = nan;
    if (fv::finite_d(fs) && fv::finite_d(K) && fv::finite_d(T) && fv::finite_d(r) &&
        fv::finite_d(qy) && fv::finite_d(sg) && fs > 0.0 && K > 0.0 && T > 0.0 && sg > 0.0 &&
        (th == 1 || th == -1)) {
      const double F = fv::forward_of(MODEL, fs, T, r, qy);
      const double D = fv::fexp_prod(-r, T);
      const double P = fv::price_at(F, K, D, sg, fv::sqrt_pos(T), th);
      gr = fv::greeks_at(MODEL, fs, K, T, r, qy, sg, th, F, D, P);
    }
    if (g.p[0]) g.p[0][i] = gr.delta;
    if (g.p[1]) g.p[1][i] = gr.gamma;
    if (g.p[2]) g.p[2][i] = gr.vega;
    if (g.p[3]) g.p[3][i] = gr.theta;
    if (g.p[4]) g.p[4][i] = gr.rho;
  }
}

// ------------------------------------------------------------- backward
struct BwdOut {
  double* p[6];
};

template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_iv_backward(KQuotes q, const double* __restrict__ sigma,
                              const double* __restrict__ gsig, BwdOut o, int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double P = ld(q.price, i), fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i),
                 r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const double sg = sigma[i], gs = gsig[i];
    const int th = ldflag(q, i);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (fv::finite_d(sg) && sg > 0.0 && fv::finite_d(fs) && fv::finite_d(K) &&
        fv::finite_d(T) && fs > 0.0 && K > 0.0 && T > 0.0) {
      const IvGrad d = fv::iv_gradient(MODEL, fs, K, T, r, qy, sg, th, P);
      if (fv::finite_d(d.dP)) {
        v[0] = gs * d.dP;
        v[1] = gs * d.dfs;
        v[2] = gs * d.dK;
        v[3] = gs * d.dT;
        v[4] = gs * d.dr;
        v[5] = gs * d.dq;
      }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (o.p[j]) o.p[j][i] = v[j];
  }
}

// ------------------------------------------------------------- price adjoint
template <int MODEL>
__global__ __launch_bounds__(kMaxBlock) void k_price_backward(KQuotes q, fv_arg sigma,
                                                              const double* __restrict__ gp,
                                                              BwdOut o, int qpt) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * qpt + threadIdx.x;
  for (int k = 0; k < qpt; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i >= q.n) return;
    const double fs = ld(q.fs, i), K = ld(q.K, i), T = ld(q.T, i), r = ld(q.r, i);
    const double qy = MODEL == fv::kBlackScholesMerton ? ld(q.q, i) : 0.0;
    const double sg = ld(sigma, i), g = gp[i];
    const int th = ldflag(q, i);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (fv::finite_d(fs) && fv::finite_d(K) && fv::finite_d(T) && fv::finite_d(r) &&
        fv::finite_d(qy) && fv::finite_d(sg) && fs > 0.0 && K > 0.0 && T > 0.0 && sg > 0.0 &&
        (th == 1 || th == -1)) {
      const double F = fv::forward_of(MODEL, fs, T, r, qy);
      const double D = fv::fexp_prod(-r, T);
      const double P = fv::price_at(F, K, D, sg, fv::sqrt_pos(T), th);
      const fv::PricePartials pp = fv::price_partials(MODEL, fs, K, T, r, qy, sg, th, F, D, P);
      v[0] = g * pp.dfs;
      v[1] = g * pp.dK;
      v[2] = g * pp.dT;
      v[3] = g * pp.dr;
      v[4] = g * pp.dq;
      v[5] = g * pp.dsigma;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (o.p[j]) o.p[j][i] = v[j];
  }
}

// ------------------------------------------------------------- chains
struct KChains {
  int64_t n_chains, n_mat, n;
  const int64_t* chain_mat_off;
  const int64_t* mat_quote_off;
  const double *F, *r, *T, *price, *K;
  const int8_t* flag;
  int hsteps;
};

// Ragged-chain kernel: one launch over the CSR offsets, one wave per two
// consecutive 64-quote slices (one coalesced 512-byte load per field and
// slice).  The wave finds the maturity and chain of its first quote by two
// 64-ary searches and every lane those of its two quotes from the next
// maturity and chain starts, for both slices before it solves either: only
// the second slice's maturity and chain indices stay live across the first
// solve, and the location is paid once per 128 quotes (four slices per
// wave were no faster, one was 2% slower).  The Halley path compacts the
// lanes that fail its convergence check into an LDS queue (wave ballots, as
// the flat Halley kernel does; two entries per thread) and the workgroup
// bisects the packed queue afterwards.
struct ChainPending {
  int64_t i;
  int32_t m, cc;  // maturity and chain of quote i
  double lo, hi;
};

template <int SOLVER>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(FV_CHAINS_WAVES_PER_EU))) void k_iv_chains(
    KChains c, double* __restrict__ sig_out, uint8_t* __restrict__ st_out) {
  constexpr bool kHalley = SOLVER == FV_SOLVER_HALLEY;
  extern __shared__ unsigned char smem_raw[];
  ChainPending* queue = reinterpret_cast<ChainPending*>(smem_raw);
  __shared__ int qcount;
  if (kHalley) {
    if (threadIdx.x == 0) qcount = 0;
    __syncthreads();
  }
  // two consecutive 64-quote slices per wave, both located before either is
  // solved (the second location reuses the first's window of starts)
  const int64_t w0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 128;
  const int lane = (int)__lane_id();
  int64_t ms[2] = {0, 0}, cs[2] = {0, 0};
  const bool any = w0 < c.n;  // wave-uniform
  if (any) {
    fv::ChainCursor cur;
    cur.init(c.mat_quote_off, c.n_mat, c.chain_mat_off, c.n_chains, w0);
    cur.slice(w0, min(w0 + 63, c.n - 1), w0 + lane, ms[0], cs[0]);
    if (w0 + 64 < c.n) cur.slice(w0 + 64, min(w0 + 127, c.n - 1), w0 + 64 + lane, ms[1], cs[1]);
  }
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int64_t i = w0 + 64 * sl + lane;
    const int64_t m = ms[sl], cc = cs[sl];
    bool fail = false;
    fv::HalleyState hs;
    hs.lo = 0.0;
    hs.hi = 0.0;
    if (any && i < c.n) {
      const double F = c.F[cc], r = c.r[cc], T = c.T[m];
      const double P = c.price[i], K = c.K[i];
      const int th = c.flag[i];
      const Reduced rd = fv::reduce_quote(fv::kBlack76, P, F, K, T, r, 0.0, th);
      uint8_t st = rd.status;
      double sg = st == fv::kQAtIntrinsic ? 0.0 : __builtin_nan("");
      if (st == fv::kQOk) {
        if (!kHalley) {
          const LbrResult res = fv::lbr_solve(rd.x, rd.beta, rd.bmax, rd.lnb, kLbrMinSteps,
                                              kLbrMaxSteps, kLbrStepTol);
          sg = res.s * rd.isqrtT;
          if (!res.converged) st = fv::kQNotConverged;
        } else {
          hs = fv::halley_solve(rd.x, rd.beta, rd.bmax, rd.lnb, c.hsteps);
          sg = hs.s * rd.isqrtT;
          fail = !hs.converged;
        }
      }
      if (!fail) {
        sig_out[i] = sg;
        if (st_out) st_out[i] = st;
      }
    }
    if (kHalley) {
      // wave-level compaction of the failing lanes into the LDS queue
      const uint64_t mask = __ballot(fail);
      if (mask) {
        int wbase = 0;
        const int cnt = __popcll(mask);
        const unsigned first = __ffsll((unsigned long long)mask) - 1;
        if (lane == (int)first) wbase = atomicAdd(&qcount, cnt);
        wbase = __shfl(wbase, first);
        if (fail) {
          const int slot = wbase + __popcll(mask & lanemask_lt());
          queue[slot].i = i;
          queue[slot].m = (int32_t)m;
          queue[slot].cc = (int32_t)cc;
          queue[slot].lo = hs.lo;
          queue[slot].hi = hs.hi;
        }
      }
    }
  }
  if (!kHalley) return;
  __syncthreads();
  // bisection fallback over the packed queue: every lane of a wave works
  const int nq = qcount;
  for (int j = threadIdx.x; j < nq; j += blockDim.x) {
    const int64_t iq = queue[j].i;
    const int64_t mq = queue[j].m, cq = queue[j].cc;
    const Reduced rd = fv::reduce_quote(fv::kBlack76, c.price[iq], c.F[cq], c.K[iq], c.T[mq],
                                        c.r[cq], 0.0, c.flag[iq]);
    const double s =
        fv::bisection_solve(rd.x, rd.beta, rd.bmax, rd.lnb, queue[j].lo, queue[j].hi, kBisectTol);
    sig_out[iq] = s * rd.isqrtT;
    if (st_out) st_out[iq] = fv::kQOk;
  }
}

// ------------------------------------------------------------- normalised b
__global__ void k_normalised_black(int64_t n, const double* __restrict__ x,
                                   const double* __restrict__ s, const int8_t* __restrict__ fl,
                                   double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], si = s[i];
  const int th = fl ? (int)fl[i] : 1;
  // out-of-the-money side by parity: b(x, s, th) = b(-|x|, s) + intrinsic
  const double xo = -fabs(xi);
  const double bmax = exp(0.5 * xo);
  const fv::NBlack nb = fv::normalised_black_t<0, true>(xo, si, bmax);
  double b = nb.b;
  // in the money: add the intrinsic th (e^{x/2} - e^{-x/2}) = th 2 sinh(x/2),
  // from expm1 so that small |x| keeps its relative precision
  if (th * xi > 0.0) b += th * (expm1(0.5 * xi) - expm1(-0.5 * xi));
  out[i] = b;
}

// binary32 copies of the autotuner's quotes (price, S, K, T, r, q, in that
// order, n floats each)
__global__ void k_tune_to_f32(int64_t n, const double* __restrict__ P, const double* __restrict__ S,
                              const double* __restrict__ K, const double* __restrict__ T,
                              const double* __restrict__ r, const double* __restrict__ q,
                              float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (float)P[i];
  out[n + i] = (float)S[i];
  out[2 * n + i] = (float)K[i];
  out[3 * n + i] = (float)T[i];
  out[4 * n + i] = (float)r[i];
  out[5 * n + i] = (float)q[i];
}

// ------------------------------------------------------------- autotune inputs
// Synthetic in-range quotes for timing candidate launch shapes: a
// counter-based generator (the splitmix64 output function of Steele, Lea &
// Flood, OOPSLA 2014) drives the same distributions as the wide-wing
// Black-Scholes-Merton workload (z~U[-6,6], sigma~logU[0.01,3],
// T~logU[1/365,5], r~U[-0.01,0.08], q~U[0,0.05], S = 100).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double unif(uint64_t key) {
  return (double)(splitmix64(key) >> 11) * 0x1.0p-53;
}

__global__ void k_tune_quotes(int64_t n, double* S, double* K, double* T, double* r,
                              double* q, double* sig, int8_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t b = (uint64_t)i * 8;
  const double z = -6.0 + 12.0 * unif(b);
  const double sg = exp(log(0.01) + unif(b + 1) * log(300.0));
  const double Ti = exp(log(1.0 / 365.0) + unif(b + 2) * log(5.0 * 365.0));
  const double ri = -0.01 + 0.09 * unif(b + 3);
  const double qi = 0.05 * unif(b + 4);
  const double F = 100.0 * exp((ri - qi) * Ti);
  S[i] = 100.0;
  K[i] = F * exp(-z * sg * sqrt(Ti));
  T[i] = Ti;
  r[i] = ri;
  q[i] = qi;
  sig[i] = sg;
  flag[i] = unif(b + 5) < 0.5 ? 1 : -1;
}

// Ragged structure for timing the chain kernel: every maturity holds
// `per_mat` quotes and every chain `mats` maturities; per-chain F = 100 and
// r, per-maturity T taken from the flat synthetic quotes.
__global__ void k_tune_chains(int64_t n_chains, int64_t n_mat, int64_t n, int mats,
                              int per_mat, const double* Tq, const double* rq, int64_t* cmo,
                              int64_t* mqo, double* F, double* r, double* T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_chains) cmo[i] = i * mats;
  if (i <= n_mat) mqo[i] = i * per_mat;
  if (i < n_chains) {
    F[i] = 100.0;
    r[i] = rq[i * mats * per_mat];
  }
  if (i < n_mat) T[i] = Tq[i * per_mat];
  (void)n;
}

// Per-quote T and r of the ragged structure (to price its quotes).
__global__ void k_tune_expand(int64_t n, int mats, int per_mat, const double* cT,
                              const double* cr, double* Te, double* re) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Te[i] = cT[i / per_mat];
  re[i] = cr[i / ((int64_t)per_mat * mats)];
}

// ------------------------------------------------------------- host side
int fail(int code, const std::string& msg) { return fvh::fail(code, msg); }

struct LaunchShape {
  int block, qpt;
};
// Defaults from timing sweeps on MI355X (the wide-wing 10M-quote batch for
// the solvers); fv_autotune re-derives them for other shapes of work.
LaunchShape g_shape[FV_KERNEL_COUNT] = {
    {256, 2},  // price
    {64, 1},   // IV LBR
    {128, 4},  // IV Halley
    {256, 1},  // Greeks
    {128, 4},  // backward
    {128, 8},  // chains
    {128, 4},  // IV Halley, binary32
};

bool valid_shape(int block, int qpt) {
  return block >= 64 && block <= kMaxBlock && block % 64 == 0 && qpt >= 1 && qpt <= 16;
}

// Dynamic LDS a kernel family needs per workgroup at a shape: the Halley
// paths' queue of failed lanes (one entry per quote of the workgroup); no
// other family uses dynamic LDS.  Shapes above kMaxQueueBytes are refused.
constexpr size_t kMaxQueueBytes = 65536;

size_t queue_bytes(int kernel, int block, int qpt) {
  if (kernel == FV_KERNEL_IV_HALLEY) return sizeof(Pending) * (size_t)block * qpt;
  if (kernel == FV_KERNEL_IV_HALLEY_F32) return sizeof(Pending32) * (size_t)block * qpt;
  if (kernel == FV_KERNEL_CHAINS) return 2 * sizeof(ChainPending) * (size_t)block;  // Halley path
  return 0;
}

// Largest batch any launch covers: every launch has at least 64 quotes per
// workgroup and at most 2^31 - 1 workgroups.
constexpr int64_t kMaxQuotes = (int64_t)0x7fffffff * 64;

int check_quotes(int model, const fv_quotes* q) {
  if (model < FV_MODEL_BLACK76 || model > FV_MODEL_BSM)
    return fail(FV_E_INVALID_ARG, "model out of range");
  if (!q) return fail(FV_E_INVALID_ARG, "quotes pointer is NULL");
  if (q->n < 0) return fail(FV_E_INVALID_ARG, "n < 0");
  if (q->n > kMaxQuotes) return fail(FV_E_INVALID_ARG, "n above 2^31 - 1 workgroups of 64");
  if (!q->flag && q->flag_value != 1 && q->flag_value != -1)
    return fail(FV_E_INVALID_ARG, "broadcast flag_value must be +1 or -1");
  return FV_OK;
}

// Maximum Halley steps before a quote goes to the bisection fallback
// (fv_set_halley_steps); read by every launch of a Halley kernel.
std::atomic<int> g_halley_steps{kHalleySteps};

KQuotes to_k(const fv_quotes* q) {
  KQuotes k;
  k.n = q->n;
  k.price = q->price;
  k.fs = q->fs;
  k.K = q->K;
  k.T = q->T;
  k.r = q->r;
  k.q = q->q;
  k.flag = q->flag;
  k.flag_value = q->flag_value;
  k.hsteps = g_halley_steps.load(std::memory_order_relaxed);
  return k;
}

dim3 grid_for(int64_t n, const LaunchShape& sh) {
  const int64_t per = (int64_t)sh.block * sh.qpt;
  return dim3((unsigned)((n + per - 1) / per));
}

int launched(const char* what) { return fvh::launched(what); }

int device_cus() {
  static int cache[64];  // per device ordinal; 0 = not yet queried
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < 64 && cache[dev] > 0) return cache[dev];
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 256;
  if (dev >= 0 && dev < 64) cache[dev] = cus;
  return cus;
}

// ---------------------------------------------------------- tuning table
// fv_autotune's results per (kernel family, model, size class of the batch);
// a launch uses the entry of its class, as measured, when there is one.
constexpr int kModels = 3;
constexpr int kBuckets = 7;
struct Tuned {
  int block, qpt;  // block == 0: not tuned
  float ms;        // the winning candidate's time when it was measured
};
Tuned g_tuned[FV_KERNEL_COUNT][kModels][kBuckets];
// while fv_autotune times a candidate, launches of that family take it as is
int g_tuning_kernel = -1;
LaunchShape g_tuning_shape = {0, 0};

// Size class of a batch of n >= 1 quotes: 0 below 2^14, then one class per
// factor of 4 ([2^14, 2^16) is 1, ...), 6 from 2^24 up.
int bucket_of(int64_t n) {
  int lg = 0;
  while (lg < 62 && ((int64_t)1 << (lg + 1)) <= n) ++lg;
  if (lg < 14) return 0;
  return std::min(kBuckets - 1, (lg - 14) / 2 + 1);
}

// The shape a launch of n quotes of `kernel` under `model` uses: a tuned
// entry of its size class if there is one, else the configured shape,
// narrowed for a batch too small to keep every SIMD busy: quotes per thread
// halve until the launch has at least 8 waves per SIMD (32 per CU; fewer,
// longer waves leave SIMDs idle at the end), and the workgroup drops to one
// wave if there is still less than one workgroup per CU.  Results never
// depend on the shape.
LaunchShape shape_for(int kernel, int model, int64_t n) {
  if (kernel == g_tuning_kernel) return g_tuning_shape;
  const Tuned& t = g_tuned[kernel][model][bucket_of(n > 0 ? n : 1)];
  if (t.block) return LaunchShape{t.block, t.qpt};
  LaunchShape sh = g_shape[kernel];
  const int64_t cus = device_cus();
  auto waves = [n](const LaunchShape& t) {
    return (n + (int64_t)t.block * t.qpt - 1) / ((int64_t)t.block * t.qpt) * (t.block / 64);
  };
  while (sh.qpt > 1 && waves(sh) < 32 * cus) sh.qpt = (sh.qpt + 1) / 2;
  if ((n + sh.block - 1) / sh.block < cus) sh.block = 64;
  return sh;
}

// Architecture name of the current device (hipDeviceProp_t::gcnArchName,
// e.g. "gfx950:sramecc+:xnack-"), the key a tuning file is valid for.
int device_arch(std::string* out) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(FV_E_HIP, "no HIP device to read the architecture of");
  *out = prop.gcnArchName;
  return FV_OK;
}

// Value of the integer field "key" inside [b, e) of a tuning file's text.
bool int_field(const std::string& t, size_t b, size_t e, const char* key, long* v) {
  const std::string k = std::string("\"") + key + "\"";
  const size_t at = t.find(k, b);
  if (at == std::string::npos || at >= e) return false;
  size_t i = at + k.size();
  while (i < e && (t[i] == ' ' || t[i] == ':')) ++i;
  char* endp = nullptr;
  const long x = strtol(t.c_str() + i, &endp, 10);
  if (endp == t.c_str() + i) return false;
  *v = x;
  return true;
}

// Reads a tuning file written by fv_tuning_save into `table` (all entries
// validated; nothing is returned on any error) and its "arch" string.
int parse_tuning(const char* path, std::string* text, std::string* arch,
                 Tuned (*table)[kModels][kBuckets]) {
  FILE* f = fopen(path, "r");
  if (!f) return fail(FV_E_INVALID_ARG, std::string("cannot read ") + path);
  char buf[4096];
  size_t got;
  text->clear();
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0 && text->size() < (1u << 20))
    text->append(buf, got);
  fclose(f);
  const std::string& t = *text;
  auto bad = [&](const char* why) {
    return fail(FV_E_INVALID_ARG, std::string("tuning file ") + path + ": " + why);
  };
  if (t.find("\"format\": \"fastvol-tuning\"") == std::string::npos) return bad("not a tuning file");
  long version = 0;
  if (!int_field(t, 0, t.size(), "version", &version) || version != 1)
    return bad("unsupported version");
  const size_t a = t.find("\"arch\": \"");
  if (a == std::string::npos) return bad("no arch");
  const size_t a0 = a + 9, a1 = t.find('"', a0);
  if (a1 == std::string::npos || a1 == a0) return bad("no arch");
  *arch = t.substr(a0, a1 - a0);
  size_t pos = t.find("\"entries\"");
  if (pos == std::string::npos) return bad("no entries");
  memset(table, 0, sizeof(Tuned) * FV_KERNEL_COUNT * kModels * kBuckets);
  while ((pos = t.find('{', pos)) != std::string::npos) {
    const size_t end = t.find('}', pos);
    if (end == std::string::npos) return bad("unterminated entry");
    long k, m, b, blk, qq;
    if (!int_field(t, pos, end, "kernel", &k) || !int_field(t, pos, end, "model", &m) ||
        !int_field(t, pos, end, "bucket", &b) || !int_field(t, pos, end, "block", &blk) ||
        !int_field(t, pos, end, "qpt", &qq))
      return bad("entry without kernel, model, bucket, block or qpt");
    if (k < 0 || k >= FV_KERNEL_COUNT || m < 0 || m >= kModels || b < 0 || b >= kBuckets)
      return bad("entry out of range");
    // range-checked before the narrowing to int
    if (blk < 1 || blk > 1 << 16 || qq < 1 || qq > 1 << 16) return bad("invalid launch shape");
    if (!valid_shape((int)blk, (int)qq) || queue_bytes((int)k, (int)blk, (int)qq) > kMaxQueueBytes)
      return bad("invalid launch shape");
    float ms = 0.0f;
    const size_t mk = t.find("\"ms\"", pos);
    if (mk != std::string::npos && mk < end) {
      size_t i = mk + 4;
      while (i < end && (t[i] == ' ' || t[i] == ':')) ++i;
      ms = (float)strtod(t.c_str() + i, nullptr);
    }
    table[k][m][b] = Tuned{(int)blk, (int)qq, ms};
    pos = end + 1;
  }
  return FV_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int fv_version(void) { return FV_ABI_VERSION; }

const char* fv_last_error(void) { return fvh::g_last_error.c_str(); }

int fv_set_launch(int kernel, int block, int qpt) {
  if (kernel < 0 || kernel >= FV_KERNEL_COUNT) return fail(FV_E_INVALID_ARG, "kernel id");
  if (!valid_shape(block, qpt)) return fail(FV_E_INVALID_ARG, "launch shape");
  if (queue_bytes(kernel, block, qpt) > kMaxQueueBytes)
    return fail(FV_E_INVALID_ARG, "launch shape: Halley queue above 64 KiB of LDS");
  g_shape[kernel].block = block;
  g_shape[kernel].qpt = qpt;
  // an explicit shape wins over the family's tuned entries
  memset(g_tuned[kernel], 0, sizeof(g_tuned[kernel]));
  return FV_OK;
}

int fv_set_halley_steps(int steps) {
  if (steps < 1 || steps > kMaxHalleySteps)
    return fail(FV_E_INVALID_ARG, "Halley steps outside [1, 64]");
  g_halley_steps.store(steps, std::memory_order_relaxed);
  return FV_OK;
}

int fv_get_halley_steps(void) { return g_halley_steps.load(std::memory_order_relaxed); }

int fv_get_launch(int kernel, int* block, int* qpt) {
  if (kernel < 0 || kernel >= FV_KERNEL_COUNT || !block || !qpt)
    return fail(FV_E_INVALID_ARG, "kernel id or NULL output");
  *block = g_shape[kernel].block;
  *qpt = g_shape[kernel].qpt;
  return FV_OK;
}

int fv_price(int model, const fv_quotes* q, fv_arg sigma, double* price_out, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  if (!price_out) return fail(FV_E_INVALID_ARG, "price_out is NULL");
  const LaunchShape sh = shape_for(FV_KERNEL_PRICE, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_price<0><<<grid, block, 0, s>>>(k, sigma, price_out, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_price<1><<<grid, block, 0, s>>>(k, sigma, price_out, sh.qpt); break;
    default: k_price<2><<<grid, block, 0, s>>>(k, sigma, price_out, sh.qpt); break;
  }
  return launched("fv_price");
}

int fv_implied_vol(int model, int solver, const fv_quotes* q, double* sigma_out,
                   uint8_t* status_out, double* const* greeks_out, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (solver != FV_SOLVER_LBR && solver != FV_SOLVER_HALLEY)
    return fail(FV_E_INVALID_ARG, "solver out of range");
  if (q->n == 0) return FV_OK;
  if (!sigma_out) return fail(FV_E_INVALID_ARG, "sigma_out is NULL");
  GreekOut g;
  g.any = 0;
  for (int j = 0; j < 5; ++j) {
    g.p[j] = greeks_out ? greeks_out[j] : nullptr;
    g.any |= g.p[j] != nullptr;
  }
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  // every per-quote field an array (q only matters for Black-Scholes-Merton)
  const bool arr = q->price.ptr && q->fs.ptr && q->K.ptr && q->T.ptr && q->r.ptr && q->flag &&
                   (model != FV_MODEL_BSM || q->q.ptr);
  if (solver == FV_SOLVER_LBR) {
    const LaunchShape sh = shape_for(FV_KERNEL_IV_LBR, model, q->n);
    const dim3 grid = grid_for(q->n, sh), block(sh.block);
#define FV_LBR(M, G)                                                                   \
  (arr ? k_iv_lbr<M, G, true><<<grid, block, 0, s>>>(k, sigma_out, status_out, g, sh.qpt) \
       : k_iv_lbr<M, G, false><<<grid, block, 0, s>>>(k, sigma_out, status_out, g, sh.qpt))
    switch (model * 2 + (g.any ? 1 : 0)) {
      case 0: FV_LBR(0, false); break;
      case 1: FV_LBR(0, true); break;
      case 2: FV_LBR(1, false); break;
      case 3: FV_LBR(1, true); break;
      case 4: FV_LBR(2, false); break;
      default: FV_LBR(2, true); break;
    }
#undef FV_LBR
    return launched("fv_implied_vol(LBR)");
  }
  const LaunchShape sh = shape_for(FV_KERNEL_IV_HALLEY, model, q->n);
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  const size_t lds = sizeof(Pending) * (size_t)sh.block * sh.qpt;
#define FV_HAL(M, G)                                                                    \
  (arr ? k_iv_halley<M, G, true><<<grid, block, lds, s>>>(k, sigma_out, status_out, g, sh.qpt) \
       : k_iv_halley<M, G, false><<<grid, block, lds, s>>>(k, sigma_out, status_out, g, sh.qpt))
  switch (model * 2 + (g.any ? 1 : 0)) {
    case 0: FV_HAL(0, false); break;
    case 1: FV_HAL(0, true); break;
    case 2: FV_HAL(1, false); break;
    case 3: FV_HAL(1, true); break;
    case 4: FV_HAL(2, false); break;
    default: FV_HAL(2, true); break;
  }
#undef FV_HAL
  return launched("fv_implied_vol(Halley)");
}

int fv_implied_vol_f32(int model, const fv_quotes_f32* q, float* sigma_out,
                       uint8_t* status_out, void* stream) {
  if (model < FV_MODEL_BLACK76 || model > FV_MODEL_BSM)
    return fail(FV_E_INVALID_ARG, "model out of range");
  if (!q) return fail(FV_E_INVALID_ARG, "quotes pointer is NULL");
  if (q->n < 0) return fail(FV_E_INVALID_ARG, "n < 0");
  if (q->n > kMaxQuotes) return fail(FV_E_INVALID_ARG, "n above 2^31 - 1 workgroups of 64");
  if (!q->flag && q->flag_value != 1 && q->flag_value != -1)
    return fail(FV_E_INVALID_ARG, "broadcast flag_value must be +1 or -1");
  if (q->n == 0) return FV_OK;
  if (!sigma_out) return fail(FV_E_INVALID_ARG, "sigma_out is NULL");
  KQuotes32 k;
  k.n = q->n;
  k.price = q->price;
  k.fs = q->fs;
  k.K = q->K;
  k.T = q->T;
  k.r = q->r;
  k.q = q->q;
  k.flag = q->flag;
  k.flag_value = q->flag_value;
  k.hsteps = g_halley_steps.load(std::memory_order_relaxed);
  const LaunchShape sh = shape_for(FV_KERNEL_IV_HALLEY_F32, model, q->n);
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  const size_t lds = sizeof(Pending32) * (size_t)sh.block * sh.qpt;
  hipStream_t s = (hipStream_t)stream;
  switch (model) {
    case FV_MODEL_BLACK76: k_iv_halley32<0><<<grid, block, lds, s>>>(k, sigma_out, status_out, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_iv_halley32<1><<<grid, block, lds, s>>>(k, sigma_out, status_out, sh.qpt); break;
    default: k_iv_halley32<2><<<grid, block, lds, s>>>(k, sigma_out, status_out, sh.qpt); break;
  }
  return launched("fv_implied_vol_f32");
}

int fv_greeks(int model, const fv_quotes* q, fv_arg sigma, double* delta, double* gamma,
              double* vega, double* theta, double* rho, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  GreekOut g;
  g.p[0] = delta; g.p[1] = gamma; g.p[2] = vega; g.p[3] = theta; g.p[4] = rho;
  g.any = 1;
  if (!delta && !gamma && !vega && !theta && !rho) return FV_OK;
  const LaunchShape sh = shape_for(FV_KERNEL_GREEKS, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_greeks<0><<<grid, block, 0, s>>>(k, sigma, g, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_greeks<1><<<grid, block, 0, s>>>(k, sigma, g, sh.qpt); break;
    default: k_greeks<2><<<grid, block, 0, s>>>(k, sigma, g, sh.qpt); break;
  }
  return launched("fv_greeks");
}

int fv_implied_vol_backward(int model, const fv_quotes* q, const double* sigma,
                            const double* grad_sigma, double* g_price, double* g_fs,
                            double* g_K, double* g_T, double* g_r, double* g_q, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  if (!sigma || !grad_sigma) return fail(FV_E_INVALID_ARG, "sigma or grad_sigma is NULL");
  BwdOut o;
  o.p[0] = g_price; o.p[1] = g_fs; o.p[2] = g_K; o.p[3] = g_T; o.p[4] = g_r; o.p[5] = g_q;
  const LaunchShape sh = shape_for(FV_KERNEL_BACKWARD, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_iv_backward<0><<<grid, block, 0, s>>>(k, sigma, grad_sigma, o, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_iv_backward<1><<<grid, block, 0, s>>>(k, sigma, grad_sigma, o, sh.qpt); break;
    default: k_iv_backward<2><<<grid, block, 0, s>>>(k, sigma, grad_sigma, o, sh.qpt); break;
  }
  return launched("fv_implied_vol_backward");
}

int fv_price_backward(int model, const fv_quotes* q, fv_arg sigma, const double* grad_price,
                      double* g_fs, double* g_K, double* g_T, double* g_r, double* g_q,
                      double* g_sigma, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  if (!grad_price) return fail(FV_E_INVALID_ARG, "grad_price is NULL");
  BwdOut o;
  o.p[0] = g_fs; o.p[1] = g_K; o.p[2] = g_T; o.p[3] = g_r; o.p[4] = g_q; o.p[5] = g_sigma;
  const LaunchShape sh = shape_for(FV_KERNEL_BACKWARD, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_price_backward<0><<<grid, block, 0, s>>>(k, sigma, grad_price, o, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_price_backward<1><<<grid, block, 0, s>>>(k, sigma, grad_price, o, sh.qpt); break;
    default: k_price_backward<2><<<grid, block, 0, s>>>(k, sigma, grad_price, o, sh.qpt); break;
  }
  return launched("fv_price_backward");
}

int fv_lbr_trace(int model, const fv_quotes* q, uint32_t* path_out, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  if (!path_out) return fail(FV_E_INVALID_ARG, "path_out is NULL");
  const LaunchShape sh = shape_for(FV_KERNEL_IV_LBR, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_lbr_trace<0><<<grid, block, 0, s>>>(k, path_out, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_lbr_trace<1><<<grid, block, 0, s>>>(k, path_out, sh.qpt); break;
    default: k_lbr_trace<2><<<grid, block, 0, s>>>(k, path_out, sh.qpt); break;
  }
  return launched("fv_lbr_trace");
}

int fv_halley_trace(int model, const fv_quotes* q, uint32_t* steps_out, void* stream) {
  int rc = check_quotes(model, q);
  if (rc) return rc;
  if (q->n == 0) return FV_OK;
  if (!steps_out) return fail(FV_E_INVALID_ARG, "steps_out is NULL");
  const LaunchShape sh = shape_for(FV_KERNEL_IV_LBR, model, q->n);
  const KQuotes k = to_k(q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid = grid_for(q->n, sh), block(sh.block);
  switch (model) {
    case FV_MODEL_BLACK76: k_halley_trace<0><<<grid, block, 0, s>>>(k, steps_out, sh.qpt); break;
    case FV_MODEL_BLACK_SCHOLES: k_halley_trace<1><<<grid, block, 0, s>>>(k, steps_out, sh.qpt); break;
    default: k_halley_trace<2><<<grid, block, 0, s>>>(k, steps_out, sh.qpt); break;
  }
  return launched("fv_halley_trace");
}

int fv_implied_vol_chains(int solver, const fv_chains* c, double* sigma_out,
                          uint8_t* status_out, void* stream) {
  if (!c) return fail(FV_E_INVALID_ARG, "chains pointer is NULL");
  if (solver != FV_SOLVER_LBR && solver != FV_SOLVER_HALLEY)
    return fail(FV_E_INVALID_ARG, "solver out of range");
  if (c->n_chains < 0 || c->n_maturities < 0 || c->n_quotes < 0)
    return fail(FV_E_INVALID_ARG, "negative size");
  if (c->n_quotes == 0) return FV_OK;
  if (c->n_quotes > kMaxQuotes) return fail(FV_E_INVALID_ARG, "n_quotes above 2^31 - 1 workgroups of 64");
  if (c->n_maturities > 0x7fffffff || c->n_chains > 0x7fffffff)
    return fail(FV_E_INVALID_ARG, "more than 2^31 - 1 maturities or chains");
  if (c->n_chains == 0 || c->n_maturities == 0)
    return fail(FV_E_INVALID_ARG, "quotes without chains or maturities");
  if (!c->chain_mat_off || !c->mat_quote_off || !c->F || !c->r || !c->T || !c->price ||
      !c->K || !c->flag || !sigma_out)
    return fail(FV_E_INVALID_ARG, "NULL chain array");
  KChains k;
  k.n_chains = c->n_chains;
  k.n_mat = c->n_maturities;
  k.n = c->n_quotes;
  k.chain_mat_off = c->chain_mat_off;
  k.mat_quote_off = c->mat_quote_off;
  k.F = c->F;
  k.r = c->r;
  k.T = c->T;
  k.price = c->price;
  k.K = c->K;
  k.flag = c->flag;
  k.hsteps = g_halley_steps.load(std::memory_order_relaxed);
  const LaunchShape sh = shape_for(FV_KERNEL_CHAINS, FV_MODEL_BLACK76, k.n);
  // one wave per 64 consecutive quotes, blockDim/64 waves per workgroup; the
  // quote count is capped (kMaxQuotes) so that the grid fits
  const int64_t n_blocks = (k.n + 2 * sh.block - 1) / (2 * sh.block);
  const dim3 grid((unsigned)n_blocks), block(sh.block);
  hipStream_t s = (hipStream_t)stream;
  if (solver == FV_SOLVER_LBR)
    k_iv_chains<FV_SOLVER_LBR><<<grid, block, 0, s>>>(k, sigma_out, status_out);
  else
    k_iv_chains<FV_SOLVER_HALLEY><<<grid, block, 2 * sizeof(ChainPending) * (size_t)sh.block, s>>>(
        k, sigma_out, status_out);
  return launched("fv_implied_vol_chains");
}

int fv_normalised_black(int64_t n, const double* x, const double* s, const int8_t* flag,
                        double* out, void* stream) {
  if (n < 0) return fail(FV_E_INVALID_ARG, "n < 0");
  if (n == 0) return FV_OK;
  if (!x || !s || !out) return fail(FV_E_INVALID_ARG, "NULL array");
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  k_normalised_black<<<grid, block, 0, (hipStream_t)stream>>>(n, x, s, flag, out);
  return launched("fv_normalised_black");
}

int fv_autotune(int kernel, int model, int64_t n_hint, void* stream) {
  if (kernel < 0 || kernel >= FV_KERNEL_COUNT) return fail(FV_E_INVALID_ARG, "kernel id");
  if (model < FV_MODEL_BLACK76 || model > FV_MODEL_BSM)
    return fail(FV_E_INVALID_ARG, "model out of range");
  if (n_hint < 0) return fail(FV_E_INVALID_ARG, "n_hint < 0");
  // time on a batch of the requested size class: n_hint quotes, at most
  // 2^24, rounded down to whole synthetic chains (at least one group of 8)
  const int per_mat = 256, mats = 8;
  int64_t n = std::min<int64_t>(n_hint, 1 << 24);
  n = std::max<int64_t>((n / (per_mat * mats)) * (per_mat * mats), per_mat * mats);
  // the chain kernel only runs Black-76
  const int tuned_model = kernel == FV_KERNEL_CHAINS ? FV_MODEL_BLACK76 : model;
  const int bucket = bucket_of(n_hint > 0 ? n_hint : 1);
  const int64_t n_mat = n / per_mat, n_chains = n_mat / mats;
  hipStream_t s = (hipStream_t)stream;

  // scratch for this call only
  std::vector<void*> bufs;
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return p;
  };
  auto release = [&]() {
    for (void* p : bufs) (void)hipFree(p);
    bufs.clear();
  };
  double *S = (double*)alloc(n * 8), *K = (double*)alloc(n * 8), *T = (double*)alloc(n * 8),
         *r = (double*)alloc(n * 8), *q = (double*)alloc(n * 8), *sig = (double*)alloc(n * 8),
         *P = (double*)alloc(n * 8), *o1 = (double*)alloc(n * 8), *o2 = (double*)alloc(n * 8);
  int8_t* flag = (int8_t*)alloc(n);
  uint8_t* st = (uint8_t*)alloc(n);
  float* f32 = kernel == FV_KERNEL_IV_HALLEY_F32 ? (float*)alloc((size_t)6 * n * 4) : nullptr;
  int64_t *cmo = (int64_t*)alloc((n_chains + 1) * 8), *mqo = (int64_t*)alloc((n_mat + 1) * 8);
  double *cF = (double*)alloc(n_chains * 8), *cr = (double*)alloc(n_chains * 8),
         *cT = (double*)alloc(n_mat * 8);
  for (void* p : bufs)
    if (!p) {
      release();
      return fail(FV_E_HIP, "fv_autotune: device allocation failed");
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    release();
    return fail(FV_E_HIP, "fv_autotune: event creation failed");
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    release();
    return fail(FV_E_HIP, "fv_autotune: event creation failed");
  }
  const unsigned g256 = (unsigned)((n + 255) / 256);
  k_tune_quotes<<<g256, 256, 0, s>>>(n, S, K, T, r, q, sig, flag);
  k_tune_chains<<<(unsigned)((n_mat + 256) / 256), 256, 0, s>>>(n_chains, n_mat, n, mats, per_mat,
                                                              T, r, cmo, mqo, cF, cr, cT);

  fv_quotes qs;
  memset(&qs, 0, sizeof(qs));
  qs.n = n;
  qs.price.ptr = P;
  qs.fs.ptr = S;
  qs.K.ptr = K;
  qs.T.ptr = T;
  qs.r.ptr = r;
  qs.q.ptr = q;
  qs.flag = flag;
  fv_arg sa;
  sa.ptr = sig;
  sa.value = 0.0;
  fv_chains cs;
  memset(&cs, 0, sizeof(cs));
  cs.n_chains = n_chains;
  cs.n_maturities = n_mat;
  cs.n_quotes = n;
  cs.chain_mat_off = cmo;
  cs.mat_quote_off = mqo;
  cs.F = cF;
  cs.r = cr;
  cs.T = cT;
  cs.price = P;
  cs.K = K;
  cs.flag = flag;

  int rc = FV_OK;
  // input prices: the model's own prices of sigma (the chain kernel reads
  // Black-76 prices of the chain forwards)
  if (kernel == FV_KERNEL_CHAINS) {
    k_tune_expand<<<g256, 256, 0, s>>>(n, mats, per_mat, cT, cr, o1, o2);
    fv_quotes cq = qs;
    cq.fs.ptr = nullptr;
    cq.fs.value = 100.0;
    cq.T.ptr = o1;
    cq.r.ptr = o2;
    rc = fv_price(FV_MODEL_BLACK76, &cq, sa, P, stream);
  } else {
    rc = fv_price(model, &qs, sa, P, stream);
  }
  fv_quotes_f32 q32;
  memset(&q32, 0, sizeof(q32));
  if (f32) {
    k_tune_to_f32<<<g256, 256, 0, s>>>(n, P, S, K, T, r, q, f32);
    q32.n = n;
    q32.price.ptr = f32;
    q32.fs.ptr = f32 + n;
    q32.K.ptr = f32 + 2 * n;
    q32.T.ptr = f32 + 3 * n;
    q32.r.ptr = f32 + 4 * n;
    q32.q.ptr = f32 + 5 * n;
    q32.flag = flag;
  }

  auto run = [&]() -> int {
    switch (kernel) {
      case FV_KERNEL_PRICE: return fv_price(model, &qs, sa, o1, stream);
      case FV_KERNEL_IV_LBR: return fv_implied_vol(model, FV_SOLVER_LBR, &qs, o1, st, nullptr, stream);
      case FV_KERNEL_IV_HALLEY:
        return fv_implied_vol(model, FV_SOLVER_HALLEY, &qs, o1, st, nullptr, stream);
      case FV_KERNEL_GREEKS: return fv_greeks(model, &qs, sa, o1, o2, nullptr, nullptr, nullptr, stream);
      case FV_KERNEL_BACKWARD:
        return fv_implied_vol_backward(model, &qs, sig, sig, o1, o2, nullptr, nullptr, nullptr,
                                       nullptr, stream);
      case FV_KERNEL_IV_HALLEY_F32:
        return fv_implied_vol_f32(model, &q32, (float*)o1, st, stream);
      default: return fv_implied_vol_chains(FV_SOLVER_LBR, &cs, o1, st, stream);
    }
  };
  const int blocks[] = {64, 128, 256, 512};
  const int qpts[] = {1, 2, 4, 8};
  LaunchShape best = {0, 0};
  float best_ms = 1e30f;
  for (int b : blocks) {
    for (int qq : qpts) {
      if (rc != FV_OK) break;
      if (queue_bytes(kernel, b, qq) > kMaxQueueBytes) continue;
      g_tuning_kernel = kernel;
      g_tuning_shape = LaunchShape{b, qq};
      rc = run();  // warm-up
      float mn = 1e30f;
      for (int rep = 0; rep < 3 && rc == FV_OK; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) {
          rc = fail(FV_E_HIP, "fv_autotune: event record");
          break;
        }
        rc = run();
        float ms = 0.0f;
        if (rc == FV_OK && (hipEventRecord(e1, s) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = fail(FV_E_HIP, "fv_autotune: event timing");
        mn = std::min(mn, ms);
      }
      if (rc == FV_OK && mn < best_ms) {
        best_ms = mn;
        best = {b, qq};
      }
    }
  }
  g_tuning_kernel = -1;
  if (rc == FV_OK && best.block)
    g_tuned[kernel][tuned_model][bucket] = Tuned{best.block, best.qpt, best_ms};
  // best-effort cleanup: an error here cannot change the result above
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  release();
  return rc;
}

int fv_launch_shape(int kernel, int model, int64_t n, int* block, int* qpt) {
  if (kernel < 0 || kernel >= FV_KERNEL_COUNT || !block || !qpt)
    return fail(FV_E_INVALID_ARG, "kernel id or NULL output");
  if (model < FV_MODEL_BLACK76 || model > FV_MODEL_BSM)
    return fail(FV_E_INVALID_ARG, "model out of range");
  if (n < 1) return fail(FV_E_INVALID_ARG, "n < 1");
  const LaunchShape sh =
      shape_for(kernel, kernel == FV_KERNEL_CHAINS ? FV_MODEL_BLACK76 : model, n);
  *block = sh.block;
  *qpt = sh.qpt;
  return FV_OK;
}

int fv_tuning_reset(void) {
  memset(g_tuned, 0, sizeof(g_tuned));
  return FV_OK;
}

int fv_tuning_save(const char* path) {
  if (!path) return fail(FV_E_INVALID_ARG, "path is NULL");
  std::string arch;
  const int rc = device_arch(&arch);
  if (rc) return rc;
  FILE* f = fopen(path, "w");
  if (!f) return fail(FV_E_INVALID_ARG, std::string("cannot write ") + path);
  fprintf(f, "{\"format\": \"fastvol-tuning\", \"version\": 1, \"arch\": \"%s\", \"entries\": [",
          arch.c_str());
  bool first = true;
  for (int k = 0; k < FV_KERNEL_COUNT; ++k)
    for (int m = 0; m < kModels; ++m)
      for (int b = 0; b < kBuckets; ++b) {
        const Tuned& t = g_tuned[k][m][b];
        if (!t.block) continue;
        fprintf(f, "%s\n  {\"kernel\": %d, \"model\": %d, \"bucket\": %d, \"block\": %d, "
                   "\"qpt\": %d, \"ms\": %.6g}",
                first ? "" : ",", k, m, b, t.block, t.qpt, (double)t.ms);
        first = false;
      }
  fprintf(f, "\n]}\n");
  const bool ok = !ferror(f);
  fclose(f);
  return ok ? FV_OK : fail(FV_E_INVALID_ARG, std::string("write failed: ") + path);
}

int fv_tuning_load(const char* path) {
  if (!path) return fail(FV_E_INVALID_ARG, "path is NULL");
  std::string text, arch;
  Tuned table[FV_KERNEL_COUNT][kModels][kBuckets];
  int rc = parse_tuning(path, &text, &arch, table);
  if (rc) return rc;
  std::string here;
  rc = device_arch(&here);
  if (rc) return rc;
  if (arch != here)
    return fail(FV_E_UNSUPPORTED, "tuning file is for " + arch + ", this device is " + here);
  memcpy(g_tuned, table, sizeof(g_tuned));
  return FV_OK;
}

}  // extern "C"
