"""Throughput of the FP64 "Let's Be Rational" implied-volatility kernel on one
MI355X, on the 10,000,000-quote Black-Scholes-Merton wide-wing workload.

A step is one fv_implied_vol launch (LBR solver) over the whole batch with
its inputs already resident in HBM: load, validate, reduce to normalised
coordinates, four-region guess, Householder(3) steps, store sigma and status.

Prints ONE JSON line (see --help for the knobs).  The CPU-baseline leg times
the binary128 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Roofline figures of the LBR kernel on this workload, taken with rocprofv3
# from the kernel sources whose code (comments and layout left out) has the
# SHA-256 ``source_sha256`` (the summaries
# and the commands that made them are kept under profiles/):
#  * flop_per_quote: algorithmic FP64 work (FMA = 2 FLOPs, every other FP64
#    VALU instruction = 1 per lane) from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64
#    of one launch over the workload with the quotes sorted by LBR path
#    (``--census``), where no wave executes a branch another lane skipped;
#  * executed_flop_per_quote: the same count on the workload as generated
#    (divergence included);
#  * valu_per_quote: SQ_INSTS_VALU x 64 / quotes of the same sorted launch,
#    every vector instruction (compares, selects, conversions included);
#  * fetch/write_bytes_per_quote: FETCH_SIZE and WRITE_SIZE of the timed
#    launch, each divided by what the counter reads per byte of a plain
#    1 GiB device copy (``--copy-probe``) and by the quote count.
# The traffic figure is reported only while the kernel sources still hash to
# ``source_sha256``; the FLOP figure is the algorithmic count of that source.
LBR_PROFILE = {
    "source_sha256": "07506ec4e603578bce41630df4e9a1a4b067c5a208677fa6be7c9fa8ba395d60",
    "flop_per_quote": 1082.5,
    "executed_flop_per_quote": 1205.6,
    "valu_per_quote": 1038.6,
    "fetch_bytes_per_quote": 50.033,
    "write_bytes_per_quote": 9.000,
}
FP64_VECTOR_PEAK_TFLOPS = 78.6
# VALU issue capacity at the nominal clock: 256 CUs x 4 SIMDs x 16 lanes,
# one lane-instruction per lane per cycle (a wave64 instruction occupies a
# SIMD for 4 cycles) at 2.4 GHz -- the rate behind the FP64 peak, counted in
# instructions of any kind instead of FMA-weighted FLOPs
VALU_LANES = 256 * 4 * 16
NOMINAL_CLOCK_HZ = 2.4e9
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per quote: six float64 inputs + int8 flag in,
# float64 sigma + uint8 status out
BYTES_PER_QUOTE = 6 * 8 + 1 + 8 + 1
KERNEL_SOURCES = ("fv_kernels.hip", "fv_math.h", "fv_lbr.h", "fv_quote.h", "fv_coeffs.h",
                  "fv_host.h", "fv_csr.h", "fv_f32.h")


def _code_only(text: str) -> str:
    """C++ source with its comments removed and every run of white space
    made one space: what a comment or layout edit leaves unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, escapes included
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_sha256() -> str:
    """SHA-256 of the kernel sources' code (comments and layout left out)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2604_27210_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode("utf-8"))
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-ms", type=float, default=200.0,
                    help="before the warmup steps, repeat the step untimed for this long: "
                         "after an idle spell the GPU raises its clock over the first ~40 ms "
                         "of sustained load (about 100 launches of this kernel run 5-20%% "
                         "slower), and the timed steps are to measure the sustained rate; "
                         "0 disables it (the line then reports the post-idle rate)")
    ap.add_argument("--n", type=int, default=10_000_000, help="quotes per step")
    ap.add_argument("--solver", default="lbr", choices=["lbr", "halley"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="quotes of the workload the oracle solves for the CPU baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (Halley, small batch, ragged chains, "
                         "forward+backward, calibration)")
    ap.add_argument("--census", action="store_true",
                    help="instead of the bench: group the quotes by LBR path (fv_lbr_trace) and "
                         "by Halley step count (fv_halley_trace), then run each solver's "
                         "kernel on the workload as generated and with the quotes sorted, so "
                         "that FP64 instruction counters (rocprofv3 --pmc) of the sorted "
                         "launches give the algorithmic work")
    ap.add_argument("--census-steady", action="store_true",
                    help="with --census, for a run without the profiler: time each order over "
                         "20 launches after the settle phase (--settle-ms), at the sustained "
                         "clock")
    ap.add_argument("--n-sweep", action="store_true",
                    help="instead of the bench: throughput of LBR and Halley IV, pricing and "
                         "Greeks on the first N quotes of the wide workload, N = 1e3 .. 1e8 "
                         "(one JSON line per N)")
    ap.add_argument("--kernel-census", action="store_true",
                    help="instead of the bench: launch every other kernel family on its "
                         "workload three times (pricing, Greeks, the IV adjoint on the 1M "
                         "differentiation workload, ragged chains with both solvers, one "
                         "calibration step of the 500-chain problem, binary32 Halley), for "
                         "rocprofv3 counter passes")
    ap.add_argument("--clock-series", action="store_true",
                    help="instead of the bench: after 2 s of idle, 40 blocks of 50 back-to-back "
                         "LBR launches with a 2 s pause after block 20; per block the mean, "
                         "first, min and max launch time (how the clock ramps under load)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="instead of the bench: copy a 1 GiB device buffer three times "
                         "(the reference launch that scales FETCH_SIZE / WRITE_SIZE to bytes)")
    return ap.parse_args()


def make_inputs(n, torch, fv):
    from paper_2604_27210_amd import workloads as W
    wl = W.bsm_wide(n, seed=2)
    d = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    S, K, T, r, q = d(wl.fs), d(wl.K), d(wl.T), d(wl.r), d(wl.q)
    flag = d(wl.flag, torch.int8)
    # clean prices from the library's own pricer; degenerate prices for the
    # injected quotes (at / below intrinsic, above the upper bound)
    P = fv.price("bsm", S, K, T, r, d(wl.sigma_true), flag=flag, q=q)
    torch.cuda.synchronize()
    Ph = P.cpu().numpy()
    F = wl.fs * np.exp((wl.r - wl.q) * wl.T)
    D = np.exp(-wl.r * wl.T)
    call = wl.flag > 0
    intrinsic = D * np.where(call, np.maximum(F - wl.K, 0), np.maximum(wl.K - F, 0))
    upper = np.where(call, D * F, D * wl.K)
    k = wl.kind
    Ph = np.where(k == W.KIND_AT, intrinsic, Ph)
    Ph = np.where(k == W.KIND_BELOW, intrinsic - wl.pert * D * F, Ph)
    Ph = np.where(k == W.KIND_ABOVE, upper * (1 + wl.pert), Ph)
    return wl, d(Ph), S, K, T, r, q, flag


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(wl, P, sample, reps=3):
    """The oracle, untuned, on `sample` quotes strided over the workload: all
    its OpenMP threads, then one thread on every 10th of those quotes; the
    wall-clock median of `reps` runs of each."""
    import oracle
    idx = np.linspace(0, wl.n - 1, sample).astype(np.int64)
    sub = wl.take(idx)
    Ps = P[idx]
    oracle._load()
    threads = oracle.num_threads()

    def wall(fn):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    dt = wall(lambda: oracle.implied_vol("bsm", Ps, sub.fs, sub.K, sub.T, sub.r, sub.q, sub.flag))
    s1 = slice(0, None, 10)
    oracle.set_threads(1)
    try:
        dt1 = wall(lambda: oracle.implied_vol("bsm", Ps[s1], sub.fs[s1], sub.K[s1], sub.T[s1],
                                              sub.r[s1], sub.q[s1], sub.flag[s1]))
    finally:
        oracle.set_threads(threads)
    n1 = len(Ps[s1])
    return {"value": sample / dt, "unit": "implied vols/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d quotes evenly strided over the 10M-quote workload, binary128 exact "
                      "root, OpenMP over %d threads, median of %d runs %.2f s wall"
                      % (sample, threads, reps, dt),
            "single_thread_value": n1 / dt1,
            "single_thread_sample": "every 10th quote of that sample (%d), one thread, median of "
                                    "%d runs %.2f s wall" % (n1, reps, dt1),
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count()}}


HOST_LBR_SRC = r"""
#include <cstdint>
#include <omp.h>
#include "fv_quote.h"
#include "fv_lbr.h"
extern "C" {
int h_threads(void) { return omp_get_max_threads(); }
// Black-Scholes-Merton implied volatility by LBR, one quote per loop
// iteration, as the flat kernel runs it per lane
void h_iv_lbr_bsm(int64_t n, const double* P, const double* S, const double* K,
                  const double* T, const double* r, const double* q, const int8_t* flag,
                  double* sig) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const fv::Reduced rd = fv::reduce_quote(fv::kBlackScholesMerton, P[i], S[i], K[i], T[i],
                                            r[i], q[i], flag[i]);
    double sg = rd.status == fv::kQAtIntrinsic ? 0.0 : __builtin_nan("");
    if (rd.status == fv::kQOk) {
      const fv::LbrResult res = fv::lbr_solve(rd.x, rd.beta, rd.bmax, rd.lnb, 2, 4, 1e-6);
      sg = res.converged ? res.s * rd.isqrtT : __builtin_nan("");
    }
    sig[i] = sg;
  }
}
}
"""


def host_fp64_lbr(wl, P, sample, reps=3):
    """Context beside the oracle: the library's own FP64 LBR (the kernels'
    headers compiled for the host with g++ -O3 and OpenMP), on `sample`
    quotes strided over the workload, all OpenMP threads; the wall-clock
    median of `reps` runs. Timing only: nothing else calls this build."""
    import ctypes
    import subprocess
    import tempfile
    d = tempfile.mkdtemp(prefix="fv_host_lbr_")
    src, so = os.path.join(d, "h.cpp"), os.path.join(d, "libh.so")
    with open(src, "w") as f:
        f.write(HOST_LBR_SRC)
    csrc = os.path.join(ROOT, "paper_2604_27210_amd", "csrc")
    cmd = ["g++", "-O3", "-march=native", "-std=gnu++17", "-fopenmp", "-shared", "-fPIC",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + csrc, src, "-o", so]
    import shutil
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        shutil.rmtree(d, ignore_errors=True)
        return {"error": "host build failed: " + res.stderr[-300:]}
    lib = ctypes.CDLL(so)
    shutil.rmtree(d, ignore_errors=True)  # the loaded library stays mapped
    idx = np.linspace(0, wl.n - 1, sample).astype(np.int64)
    sub = wl.take(idx)
    arrs = [np.ascontiguousarray(a, dtype=np.float64)
            for a in (P[idx], sub.fs, sub.K, sub.T, sub.r, sub.q)]
    fl = np.ascontiguousarray(sub.flag, dtype=np.int8)
    sig = np.empty(sample)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    run = lambda: lib.h_iv_lbr_bsm(ctypes.c_int64(sample), *[vp(a) for a in arrs], vp(fl),
                                   vp(sig))
    run()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        ts.append(time.perf_counter() - t0)
    dt = float(np.median(ts))
    threads = int(lib.h_threads())
    return {"value": sample / dt, "unit": "implied vols/s", "cores": threads,
            "kind": "library LBR compiled for the host (g++ -O3 -march=native, OpenMP)",
            "sample": "%d quotes evenly strided over the %d-quote workload, %d threads, "
                      "median of %d runs %.3f s wall" % (sample, wl.n, threads, reps, dt)}


def _settle(torch, fn, ms=100.0):
    """Repeat fn untimed for `ms` of wall time, so that the timing after it
    sees the GPU's sustained clock rather than its ramp after host-side
    setup (see --settle-ms)."""
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(5):
            fn()
        torch.cuda.synchronize()


def _time(torch, fn, reps=10, warm=2, settle_ms=100.0):
    if settle_ms > 0:
        _settle(torch, fn, settle_ms)
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _time_cold(torch, fn, reps=10, warm=2):
    """As _time, with the caches flushed before every timed call by a
    1 GiB device write (larger than L2 plus the 256 MB Infinity Cache)."""
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        flush.fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del flush
    return float(np.median(ts))


def _graph_replay_us(torch, fn, reps=50):
    """Median time (us) of one replay of a graph that captured fn once."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up on the side stream, outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return _time(torch, g.replay, reps=reps, warm=3) * 1e3


def extras(fv, torch, main_inputs, sig_true):
    """Secondary measurements beside the headline: the Halley path on the
    same batch, pricing and Greeks on it against a plain device copy, the
    small batch's latency, ragged chains (one persistent launch vs the flat
    kernel on expanded arrays vs one launch per chain), forward+backward of
    the differentiable IV, and the hipGraph calibration loop (graph replay
    vs eager launches)."""
    from paper_2604_27210_amd import workloads as W
    from paper_2604_27210_amd.calibrate import SviCalibrator, calibrate_svi, raw_from_natural
    d = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    out = {}
    P, S, K, T, r, q, flag = main_inputs
    n = P.numel()
    # the memory-heavy paths against the HBM rate a plain device copy reaches
    # on this machine (the same bytes as the pricing call moves)
    src = torch.empty(n * 57 // 16, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    copy_ms = _time(torch, lambda: dst.copy_(src), reps=50)
    copy_gbs = 2 * src.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del src, dst
    out["hbm_device_copy_GBs"] = copy_gbs
    for name, fn, nbytes in (
            ("price_bsm", lambda: fv.price("bsm", S, K, T, r, sig_true, flag=flag, q=q), 49 + 8),
            ("greeks_bsm", lambda: fv.greeks("bsm", S, K, T, r, sig_true, flag=flag, q=q),
             49 + 40)):
        ms = _time(torch, fn, reps=50)
        gbs = nbytes * n / (ms * 1e-3) / 1e9
        out[name] = {"ms": ms, "per_s": n / ms * 1e3, "algorithmic_GBs": gbs,
                     "frac_of_device_copy": gbs / copy_gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    ms = _time(torch, lambda: fv.implied_vol("bsm", P, S, K, T, r, flag=flag, q=q, solver="halley"))
    out["halley_wide_bsm"] = {"ms": ms, "implied_vols_per_s": n / ms * 1e3}
    # the binary32 Halley path on the same quotes rounded to float32
    f32 = [x.float() for x in (P, S, K, T, r, q)]
    ms = _time(torch, lambda: fv.implied_vol_f32("bsm", f32[0], f32[1], f32[2], f32[3], f32[4],
                                                  flag=flag, q=f32[5]))
    out["halley_f32_wide_bsm"] = {"ms": ms, "implied_vols_per_s": n / ms * 1e3}
    del f32
    # small batch: launch-latency bound
    wl = W.bs_small()
    a = [d(x) for x in (wl.fs, wl.K, wl.T, wl.r)]
    fl = d(wl.flag, torch.int8)
    Ps = fv.price("bs", a[0], a[1], a[2], a[3], d(wl.sigma_true), flag=fl)
    for solver in ("lbr", "halley"):
        call = lambda: fv.implied_vol("bs", Ps, *a, flag=fl, solver=solver)
        out["bs_4096_%s_us_per_call" % solver] = _time(torch, call, reps=50) * 1e3
        out["bs_4096_%s_us_per_graph_replay" % solver] = _graph_replay_us(torch, call)
    # ragged chains
    ch = W.b76_chains()
    flat = ch.flatten()
    cd = {k: d(v, torch.int64) for k, v in (("cmo", ch.chain_mat_off), ("mqo", ch.mat_quote_off))}
    F, rc, Tm, Kq, flq = d(ch.F), d(ch.r), d(ch.T), d(ch.K), d(ch.flag, torch.int8)
    fF, fT, fr = d(flat.fs), d(flat.T), d(flat.r)
    Pc = fv.price("black76", fF, Kq, fT, fr, d(ch.sigma_true), flag=flq)
    persistent = lambda: fv.implied_vol_chains(cd["cmo"], cd["mqo"], F, rc, Tm, Pc, Kq, flq)
    ms_p = _time(torch, persistent)
    ms_pc = _time_cold(torch, persistent)
    ms_f = _time(torch, lambda: fv.implied_vol("black76", Pc, fF, Kq, fT, fr, flag=flq))
    # what a caller without the ragged call pays: gather the per-chain F, r
    # and per-maturity T to per-quote arrays on the device, then the flat call
    mat_q = d(ch.mat_of_quote(), torch.int64)
    chain_q = d(ch.chain_of_mat()[ch.mat_of_quote()], torch.int64)

    def expand_then_flat():
        eF, eT, er = F.index_select(0, chain_q), Tm.index_select(0, mat_q), rc.index_select(0, chain_q)
        return fv.implied_vol("black76", Pc, eF, Kq, eT, er, flag=flq)
    ms_ef = _time(torch, expand_then_flat)
    off = ch.mat_quote_off[ch.chain_mat_off]

    def per_chain():
        for c in range(ch.n_chains):
            lo, hi = int(off[c]), int(off[c + 1])
            fv.implied_vol("black76", Pc[lo:hi], fF[lo:hi], Kq[lo:hi], fT[lo:hi], fr[lo:hi],
                           flag=flq[lo:hi])
    ms_c = _time(torch, per_chain, reps=3, warm=1)
    out["ragged_b76_chains"] = {"n_quotes": ch.n, "n_chains": ch.n_chains, "n_maturities": ch.n_mat,
                                "persistent_ms": ms_p, "persistent_cold_ms": ms_pc,
                                "flat_expanded_ms": ms_f,
                                "expand_on_device_then_flat_ms": ms_ef,
                                "per_chain_launches_ms": ms_c,
                                "persistent_implied_vols_per_s": ch.n / ms_p * 1e3}
    # forward + backward (differentiable IV), 1M quotes
    wd = W.bsm_diff()
    x = [d(v) for v in (wd.fs, wd.K, wd.T, wd.r, wd.q)]
    fld = d(wd.flag, torch.int8)
    Pd = fv.price("bsm", x[0], x[1], x[2], x[3], d(wd.sigma_true), flag=fld, q=x[4])
    w = d(wd.extra["w"])

    def fwd_bwd():
        sig, st = fv.implied_vol("bsm", Pd, x[0], x[1], x[2], x[3], flag=fld, q=x[4])
        fv.implied_vol_backward("bsm", Pd, x[0], x[1], x[2], x[3], sig, w, flag=fld, q=x[4])
    ms_fb = _time(torch, fwd_bwd)
    ms_fw = _time(torch, lambda: fv.implied_vol("bsm", Pd, x[0], x[1], x[2], x[3], flag=fld, q=x[4]))
    # the configuration as stated: forward IV with the five Greeks fused in,
    # backward through torch.autograd to all six inputs, L = sum(w sigma)
    leaves = [t.clone().requires_grad_(True) for t in [Pd] + x]

    def fwd_bwd_autograd():
        for t in leaves:
            t.grad = None
        sig, st, gk = fv.implied_vol_autograd("bsm", *leaves[:5], flag=fld, q=leaves[5],
                                              greeks=True)
        (w * sig).sum().backward()
    ms_ag = _time(torch, fwd_bwd_autograd)
    out["bsm_1m_fwd_bwd"] = {"ms": ms_fb, "quotes_per_s": wd.n / ms_fb * 1e3,
                             "forward_only_ms": ms_fw,
                             "calls": "fv_implied_vol + fv_implied_vol_backward",
                             "autograd_with_greeks_ms": ms_ag,
                             "autograd_with_greeks_quotes_per_s": wd.n / ms_ag * 1e3}
    # calibration loop: 500 chains, 200 Adam steps, one hipGraph replay per step
    cal = W.svi_calibration(500, seed=5)
    chc = cal.chains
    mat = chc.mat_of_quote()
    chain = chc.chain_of_mat()[mat]
    th = raw_from_natural(cal.theta_true)
    # target vols: SVI(theta_true) * (1 + eps), priced and inverted on the GPU
    kq = chc.k
    a_, b_, rho_, m_, s_ = (th[:, 0], np.log1p(np.exp(th[:, 1])), np.tanh(th[:, 2]), th[:, 3],
                            np.log1p(np.exp(th[:, 4])))
    dk = kq - m_[mat]
    wv = a_[mat] + b_[mat] * (rho_[mat] * dk + np.sqrt(dk * dk + s_[mat] ** 2))
    sig_t = np.sqrt(wv / chc.T[mat]) * (1 + cal.eps)
    cF, cT, cr = d(chc.F[chain]), d(chc.T[mat]), d(chc.r[chain])
    cK, cfl = d(chc.K), d(chc.flag, torch.int8)
    Pt = fv.price("black76", cF, cK, cT, cr, d(sig_t), flag=cfl)
    iv_t, st_t = fv.implied_vol("black76", Pt, cF, cK, cT, cr, flag=cfl)
    iv_t = torch.where(st_t == 0, iv_t, torch.full_like(iv_t, float("nan")))
    args = (d(chc.chain_mat_off, torch.int64), d(chc.mat_quote_off, torch.int64), d(chc.F),
            d(chc.r), d(chc.T), cK, cfl, iv_t)
    res = {}
    # 200 untimed steps of a throw-away calibrator first (sustained clock)
    calibrate_svi(SviCalibrator(*args, raw_from_natural(cal.theta0)), 200, graph=False)
    # eager launches; one step per graph replay; ten steps per replay; the
    # whole 200-step loop as one graph
    for name, graph, k in (("eager", False, 1), ("graph", True, 1),
                           ("graph_10_steps_per_replay", True, 10),
                           ("graph_200_steps_per_replay", True, 200)):
        c = SviCalibrator(*args, raw_from_natural(cal.theta0))
        r_ = calibrate_svi(c, 200, graph=graph, steps_per_replay=k)
        ok = torch.isfinite(iv_t)
        rmse = 100 * torch.sqrt(torch.mean((c.vols()[ok] - iv_t[ok]) ** 2)).item()
        res[name] = {"steps_per_s": r_["steps_per_s"], "final_rmse_vol_points": rmse,
                     "final_loss": float(c.losses()[-1])}
    # the oracle's final RMSE on the same problem (binary128 targets, numpy
    # replay of the 200 steps), stored by tests/golden/make_svi_calibration.py
    gold_path = os.path.join(ROOT, "tests", "golden", "svi_calibration_500.json")
    with open(gold_path) as fh:
        gold = json.load(fh)
    res["oracle_final_rmse_vol_points"] = gold["final_rmse_vol_points"]
    res["graph_minus_oracle_rmse_vol_points"] = (res["graph"]["final_rmse_vol_points"]
                                                 - gold["final_rmse_vol_points"])
    out["svi_calibration_500_chains"] = dict(n_quotes=chc.n, n_maturities=chc.n_mat,
                                             steps=200, **res)
    return out


def kernel_census(fv, torch, P, S, K, T, r, q, flag, sig_true):
    """Three launches of each non-headline kernel family on its workload
    (the counter summaries read the last of each)."""
    from paper_2604_27210_amd import workloads as W
    from paper_2604_27210_amd.calibrate import SviCalibrator, raw_from_natural
    d = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    calls = {}
    calls["price_bsm_10M"] = lambda: fv.price("bsm", S, K, T, r, sig_true, flag=flag, q=q)
    calls["greeks_bsm_10M"] = lambda: fv.greeks("bsm", S, K, T, r, sig_true, flag=flag, q=q)
    f32 = [x.float() for x in (P, S, K, T, r, q)]
    calls["halley_f32_bsm_10M"] = lambda: fv.implied_vol_f32("bsm", f32[0], f32[1], f32[2], f32[3],
                                                            f32[4], flag=flag, q=f32[5])
    wd = W.bsm_diff()
    x = [d(v) for v in (wd.fs, wd.K, wd.T, wd.r, wd.q)]
    fld = d(wd.flag, torch.int8)
    Pd = fv.price("bsm", x[0], x[1], x[2], x[3], d(wd.sigma_true), flag=fld, q=x[4])
    sd, _ = fv.implied_vol("bsm", Pd, x[0], x[1], x[2], x[3], flag=fld, q=x[4])
    w = d(wd.extra["w"])
    calls["iv_backward_bsm_1M"] = lambda: fv.implied_vol_backward("bsm", Pd, x[0], x[1], x[2],
                                                                  x[3], sd, w, flag=fld, q=x[4])
    ch = W.b76_chains()
    flat = ch.flatten()
    F, rc, Tm, Kq, flq = d(ch.F), d(ch.r), d(ch.T), d(ch.K), d(ch.flag, torch.int8)
    Pc = fv.price("black76", d(flat.fs), Kq, d(flat.T), d(flat.r), d(ch.sigma_true), flag=flq)
    co, mo = d(ch.chain_mat_off, torch.int64), d(ch.mat_quote_off, torch.int64)
    for solver in ("lbr", "halley"):
        calls["chains_%s_b76_8.4M" % solver] = (
            lambda solver=solver: fv.implied_vol_chains(co, mo, F, rc, Tm, Pc, Kq, flq,
                                                        solver=solver))
    cal = W.svi_calibration(500, seed=5)
    chc = cal.chains
    mat = chc.mat_of_quote()
    chain = chc.chain_of_mat()[mat]
    cF, cT, cr, cK, cfl = (d(chc.F[chain]), d(chc.T[mat]), d(chc.r[chain]), d(chc.K),
                           d(chc.flag, torch.int8))
    Pt = fv.price("black76", cF, cK, cT, cr, d(np.full(chc.n, 0.3)), flag=cfl)
    iv_t, _ = fv.implied_vol("black76", Pt, cF, cK, cT, cr, flag=cfl)
    svi = SviCalibrator(d(chc.chain_mat_off, torch.int64), d(chc.mat_quote_off, torch.int64),
                        d(chc.F), d(chc.r), d(chc.T), cK, cfl, iv_t, raw_from_natural(cal.theta0))
    calls["svi_step_500_chains"] = svi.step
    for name, fn in calls.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        print(json.dumps({"kernel_census": name}), flush=True)


def clock_series(fv, torch, P, S, K, T, r, q, flag):
    """Launch times of the LBR kernel in blocks of 50 back-to-back launches,
    from an idle GPU, with a 2 s pause after block 20."""
    call = lambda: fv.implied_vol("bsm", P, S, K, T, r, flag=flag, q=q)
    torch.cuda.synchronize()
    time.sleep(2.0)
    t0 = time.perf_counter()
    for blk in range(40):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(50)]
        for e0, e1 in evs:
            e0.record()
            call()
            e1.record()
        torch.cuda.synchronize()
        ms = [e0.elapsed_time(e1) for e0, e1 in evs]
        print(json.dumps({"block": blk, "t_s": round(time.perf_counter() - t0, 3),
                          "mean_ms": round(float(np.mean(ms)), 4), "first_ms": round(ms[0], 4),
                          "min_ms": round(min(ms), 4), "max_ms": round(max(ms), 4)}), flush=True)
        if blk == 19:
            time.sleep(2.0)


def n_sweep(fv, torch):
    """Throughput against batch size on prefixes of one 10^8-quote draw of
    the wide BSM workload (prices from the library's pricer, no injected
    quotes): where launch latency stops dominating and where each path
    saturates the device."""
    from paper_2604_27210_amd import workloads as W
    n_max = 100_000_000
    wl = W.bsm_wide(n_max, seed=2, inject=0.0)
    d = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    S, K, T, r, q, sg = (d(x) for x in (wl.fs, wl.K, wl.T, wl.r, wl.q, wl.sigma_true))
    flag = d(wl.flag, torch.int8)
    del wl
    P = fv.price("bsm", S, K, T, r, sg, flag=flag, q=q)
    torch.cuda.synchronize()
    for n in (1_000, 10_000, 100_000, 1_000_000, 10_000_000, 100_000_000):
        a = [x[:n] for x in (P, S, K, T, r, q, sg)]
        fl = flag[:n]
        reps = 50 if n <= 1_000_000 else (10 if n <= 10_000_000 else 5)
        row = {"n_sweep": True, "n": n}
        for name, fn in (
                ("lbr", lambda: fv.implied_vol("bsm", a[0], a[1], a[2], a[3], a[4], flag=fl, q=a[5],
                                               solver="lbr")),
                ("halley", lambda: fv.implied_vol("bsm", a[0], a[1], a[2], a[3], a[4], flag=fl,
                                                  q=a[5], solver="halley")),
                ("price", lambda: fv.price("bsm", a[1], a[2], a[3], a[4], a[6], flag=fl, q=a[5])),
                ("greeks", lambda: fv.greeks("bsm", a[1], a[2], a[3], a[4], a[6], flag=fl, q=a[5]))):
            ms = _time(torch, fn, reps=reps, warm=2)
            row[name + "_ms"] = ms
            row[name + "_per_s"] = n / ms * 1e3
        print(json.dumps(row), flush=True)


def census(fv, torch, P, S, K, T, r, q, flag, steady_settle_ms=0.0):
    """Each solver's kernel on the workload as generated and with the quotes
    sorted by the work each takes (LBR: path code from fv_lbr_trace; Halley:
    step count and fallback bit from fv_halley_trace), one warm-up launch
    then five timed ones per order, no settle phase: a counter run
    (rocprofv3 --pmc) sees 6 dispatches per order and solver, and the
    sorted order's last dispatch, in which no wave executes a branch another
    of its lanes skipped, gives the algorithmic counts.

    With steady_settle_ms > 0 (a run without the profiler) each order is
    instead timed over 20 launches after that long a settle phase, so the
    times are taken at the sustained clock."""
    out = {"census": True, "n": int(P.numel()), "steady_settle_ms": steady_settle_ms}
    for solver, trace in (("lbr", fv.lbr_trace), ("halley", fv.halley_trace)):
        code = trace("bsm", P, S, K, T, r, flag=flag, q=q)
        order = torch.argsort(code.to(torch.int64))
        cs = code[order]
        args = [x.index_select(0, order).contiguous() for x in (P, S, K, T, r, q)]
        fl = flag.index_select(0, order).contiguous()
        times = {}
        for label, ins, f in (("as_generated", (P, S, K, T, r, q), flag),
                              ("sorted_by_path", args, fl)):
            run = lambda: fv.implied_vol("bsm", ins[0], ins[1], ins[2], ins[3], ins[4], flag=f,
                                         q=ins[5], solver=solver)
            if steady_settle_ms > 0:
                times[label] = _time(torch, run, reps=20, warm=3, settle_ms=steady_settle_ms)
            else:
                times[label] = _time(torch, run, reps=5, warm=1, settle_ms=0)
        c = cs.cpu().numpy().astype(np.uint32)
        solved = c != 0xFFFFFFFF
        rec = {"solved": int(solved.sum()), "distinct_paths": int(len(np.unique(c[solved]))),
               "ms_as_generated": times["as_generated"],
               "ms_sorted_by_path": times["sorted_by_path"]}
        if solver == "lbr":
            rec["region_fraction_R1_R4"] = (np.bincount(c[solved] & 3, minlength=4)
                                            / solved.sum()).round(4).tolist()
            rec["steps_fraction_2_3_4"] = (np.bincount((c[solved] >> 2) & 3, minlength=3)
                                           / solved.sum()).round(5).tolist()
        else:
            st = c[solved] & 0xFF
            rec["halley_steps_mean"] = round(float(st.mean()), 4)
            rec["halley_steps_hist_1_8"] = np.bincount(st, minlength=9)[1:].tolist()
            rec["fallback_fraction"] = round(float(((c[solved] >> 8) & 1).mean()), 6)
            # the largest step count in each wave of the as-generated order
            # (64 consecutive quotes), which the wave runs to
            cg = code.cpu().numpy().astype(np.uint32)
            m = len(cg) // 64 * 64
            w = np.where(cg[:m] == 0xFFFFFFFF, 0, cg[:m] & 0xFF).reshape(-1, 64).max(1)
            rec["wave_max_steps_mean"] = round(float(w.mean()), 4)
        out[solver] = rec
    out["launch_order"] = ["lbr as_generated", "lbr sorted_by_path", "halley as_generated",
                           "halley sorted_by_path"]
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(quotes are independent, so a multi-GPU run would shard the batch by contiguous "
              "index ranges with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2604_27210_amd as fv
    fv._native.load()
    torch.cuda.init()
    if a.n_sweep:
        n_sweep(fv, torch)
        return
    wl, P, S, K, T, r, q, flag = make_inputs(a.n, torch, fv)
    stream = torch.cuda.current_stream()
    if a.census:
        census(fv, torch, P, S, K, T, r, q, flag,
               a.settle_ms if a.census_steady else 0.0)
        return
    if a.clock_series:
        clock_series(fv, torch, P, S, K, T, r, q, flag)
        return
    if a.kernel_census:
        kernel_census(fv, torch, P, S, K, T, r, q, flag, torch.from_numpy(wl.sigma_true).cuda())
        return
    if a.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": True, "bytes_read": src.numel() * 8,
                          "bytes_written": dst.numel() * 8}), flush=True)
        return

    def step():
        return fv.implied_vol("bsm", P, S, K, T, r, flag=flag, q=q, solver=a.solver)

    # the same rate right after an idle spell (no settling), for the record
    post_idle = None
    if a.settle_ms > 0 and not a.no_extras:
        torch.cuda.synchronize()
        time.sleep(1.0)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(a.warmup + a.steps)]
        for e0, e1 in evs:
            e0.record(stream)
            step()
            e1.record(stream)
        torch.cuda.synchronize()
        post_idle = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs[a.warmup:]]))
    settle = {"ms": 0.0, "launches": 0}
    t_settle = time.perf_counter()
    while (time.perf_counter() - t_settle) * 1e3 < a.settle_ms:
        for _ in range(10):
            step()
        settle["launches"] += 10
        torch.cuda.synchronize()
    settle["ms"] = (time.perf_counter() - t_settle) * 1e3
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        sig, st = step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms = wall * 1e3 / a.steps
    avg_kernel_s = float(np.mean(kern_ms)) * 1e-3
    value = a.n / (wall / a.steps)
    st_h = st.cpu().numpy()
    counts = np.bincount(st_h, minlength=6)
    # the same call after a 1 GiB write has flushed L2 and the Infinity Cache
    kernel_ms_cold = _time_cold(torch, step, reps=5, warm=1)

    roof = None
    if a.solver == "lbr":
        ach = LBR_PROFILE["flop_per_quote"] * a.n / avg_kernel_s / 1e12
        traffic = None
        fresh = LBR_PROFILE["source_sha256"] == kernel_source_sha256()
        if fresh and LBR_PROFILE["fetch_bytes_per_quote"] is not None:
            traffic = (LBR_PROFILE["fetch_bytes_per_quote"] +
                       LBR_PROFILE["write_bytes_per_quote"]) * a.n
        roof = {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                "flop_per_quote": LBR_PROFILE["flop_per_quote"],
                # the FP64 work the launch executes on the workload as
                # generated (lanes a wave carries through branches they do
                # not take included), against the same peak: context for
                # frac, which counts the algorithmic work only
                "executed_frac": LBR_PROFILE["executed_flop_per_quote"] * a.n / avg_kernel_s / 1e12
                                 / FP64_VECTOR_PEAK_TFLOPS,
                # share of the chip's VALU issue capacity at 2.4 GHz that the
                # launch's census vector instructions fill
                "valu_issue_frac": LBR_PROFILE["valu_per_quote"] * a.n /
                                   (VALU_LANES * NOMINAL_CLOCK_HZ * avg_kernel_s),
                "kernel_ms_mean": avg_kernel_s * 1e3,
                "kernel_ms_cold": kernel_ms_cold,
                "algorithmic_hbm_GBs": BYTES_PER_QUOTE * a.n / avg_kernel_s / 1e9}
    else:
        ach = BYTES_PER_QUOTE * a.n / avg_kernel_s / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None}

    out = {
        "metric": "implied vols/sec, FP64 LBR, 10M quotes at <=1e-12 rel err",
        "value": value,
        "unit": "implied vols/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "kernel_ms_mean": float(np.mean(kern_ms)),
        "clock_settle": {"ms": settle["ms"], "launches": settle["launches"],
                         "kernel_ms_mean_post_idle": post_idle,
                         "note": "untimed steps before the warmup, until the GPU holds its "
                                 "sustained clock; kernel_ms_mean_post_idle is the timed "
                                 "window's mean when it starts after 1 s of idle"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic, seeded",
        "config": {"workload": "Black-Scholes-Merton IV, %d quotes, FP64 SoA, wide wings "
                               "(z~U[-6,6], sigma~logU[0.01,3], T~logU[1/365,5]), 1%% injected "
                               "degenerate prices" % a.n,
                   "solver": a.solver, "status_counts": counts.tolist()},
        "roofline": roof,
    }
    if not a.no_extras:
        out["extras"] = extras(fv, torch, (P, S, K, T, r, q, flag),
                               torch.from_numpy(wl.sigma_true).cuda())
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, P.cpu().numpy(), a.cpu_sample)
        out.setdefault("extras", {})["host_fp64_lbr"] = host_fp64_lbr(wl, P.cpu().numpy(), wl.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
