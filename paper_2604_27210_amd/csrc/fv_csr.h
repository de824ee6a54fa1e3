// fv_csr.h -- wave-cooperative location of quotes in CSR (offset-array)
// layouts: chain -> maturity -> quote, as the ragged-chain and calibration
// kernels read them.  Every helper here is called by all 64 lanes of a wave
// together and returns wave-uniform results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fv {

constexpr int64_t kOffEnd = INT64_MAX;

__device__ __forceinline__ int64_t ld_off(const int64_t* __restrict__ off, int64_t count,
                                          int64_t idx) {
  return idx < count ? off[idx] : kOffEnd;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Largest m in [0, count) with off[m] <= key (off non-decreasing, off[0] <=
// key): a 64-ary search, each level one load per lane at 64 evenly spaced
// candidates and a ballot, so log64(count) dependent loads instead of
// log2(count).  The loads stay below `hi` <= count; malformed (decreasing)
// offsets still shrink [lo, hi) every level.
__device__ __forceinline__ int64_t wave_locate(const int64_t* __restrict__ off, int64_t count,
                                               int64_t key) {
  const int64_t lane = __lane_id();
  int64_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) >> 6;
    const int64_t idx = lo + (lane + 1) * step;
    const bool le = idx < hi && off[idx] <= key;
    const int cnt = __popcll(__ballot(le));
    lo += (int64_t)cnt * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// The next 64 starts after `base` (lane j holds off[base + 1 + j], or kOffEnd
// past the last entry), consumed in order through a wave-uniform cursor.
struct OffWindow {
  const int64_t* off;
  int64_t count, base, v;
  int j;
  __device__ __forceinline__ void init(const int64_t* o, int64_t c, int64_t b) {
    off = o; count = c; base = b; j = 0;
    v = ld_off(off, count, base + 1 + __lane_id());
  }
  __device__ __forceinline__ int64_t peek() {
    if (j == 64) {
      base += 64;
      j = 0;
      v = ld_off(off, count, base + 1 + __lane_id());
    }
    return readlane64(v, j);
  }
  __device__ __forceinline__ void pop() { ++j; }
};

// Maturity and chain of every lane's quote as a wave walks consecutive
// 64-quote slices in increasing order (slice k covers quotes i0 .. i0 + 63,
// lane l holds quote i0 + l).  The wave finds the maturity and chain of its
// first quote by two 64-ary searches, then keeps a window of the next 64
// maturity starts and chain starts in registers: each slice reads the starts
// that fall inside it (a few wave-uniform readlanes, usually none) and every
// lane gets its maturity and chain without a search of its own.
struct ChainCursor {
  OffWindow mw, cw;
  int64_t mstart, cstart;  // maturity and chain of the current slice's first quote
  __device__ __forceinline__ void init(const int64_t* mat_quote_off, int64_t n_mat,
                                       const int64_t* chain_mat_off, int64_t n_chains,
                                       int64_t w0) {
    mstart = wave_locate(mat_quote_off, n_mat, w0);
    cstart = wave_locate(chain_mat_off, n_chains, mstart);
    mw.init(mat_quote_off, n_mat, mstart);
    cw.init(chain_mat_off, n_chains, cstart);
  }
  // The slice starting at quote i0 whose last quote is ilast; lane's quote i.
  // Returns the lane's maturity in m and chain in cc.
  __device__ __forceinline__ void slice(int64_t i0, int64_t ilast, int64_t i, int64_t& m,
                                        int64_t& cc) {
    // maturity of every lane: starts at or before i0, then those inside
    while (mw.peek() <= i0) { ++mstart; mw.pop(); }
    int64_t mm = mstart, npop = 0;
    for (int64_t b; (b = mw.peek()) <= ilast; mw.pop(), ++npop) mm += (i >= b);
    // chain of every lane, keyed by maturity
    const int64_t mlast = mstart + npop;
    while (cw.peek() <= mstart) { ++cstart; cw.pop(); }
    int64_t c = cstart, cpop = 0;
    for (int64_t b; (b = cw.peek()) <= mlast; cw.pop(), ++cpop) c += (mm >= b);
    mstart += npop;
    cstart += cpop;
    m = mm;
    cc = c;
  }
};

}  // namespace fv
