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

# Algorithmic FP64 work per quote of the LBR kernel on this workload (FMA = 2
# FLOPs), from the per-region instruction census (see profiles/).  Used for
# the roofline fraction; the measured time is what the bench reports.
LBR_FLOP_PER_QUOTE = None
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per quote: six float64 inputs + int8 flag in,
# float64 sigma + uint8 status out
BYTES_PER_QUOTE = 6 * 8 + 1 + 8 + 1


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000, help="quotes per step")
    ap.add_argument("--solver", default="lbr", choices=["lbr", "halley"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="quotes of the workload the oracle solves for the CPU baseline")
    ap.add_argument("--census", action="store_true",
                    help="instead of the bench: group the quotes by LBR path (fv_lbr_trace), "
                         "then run the LBR kernel once on the workload as generated and once "
                         "with quotes sorted by path, so that FP64 instruction counters "
                         "(rocprofv3 --pmc) of the sorted launch give the algorithmic work")
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


def cpu_baseline(wl, P, sample):
    import oracle
    idx = np.linspace(0, wl.n - 1, sample).astype(np.int64)
    sub = wl.take(idx)
    Ps = P[idx]
    oracle._load()
    t0 = time.perf_counter()
    oracle.implied_vol("bsm", Ps, sub.fs, sub.K, sub.T, sub.r, sub.q, sub.flag)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "implied vols/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d quotes evenly strided over the 10M-quote workload, binary128 exact "
                      "root, OpenMP over %d threads, %.2f s wall" % (sample, oracle.num_threads(), dt)}


def census(fv, torch, P, S, K, T, r, q, flag):
    code = fv.lbr_trace("bsm", P, S, K, T, r, flag=flag, q=q)
    order = torch.argsort(code.to(torch.int64))
    cs = code[order]
    args = [x.index_select(0, order).contiguous() for x in (P, S, K, T, r, q)]
    fl = flag.index_select(0, order).contiguous()
    times = {}
    for label, ins, f in (("as_generated", (P, S, K, T, r, q), flag), ("sorted_by_path", args, fl)):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fv.implied_vol("bsm", ins[0], ins[1], ins[2], ins[3], ins[4], flag=f, q=ins[5], solver="lbr")
        e1.record()
        torch.cuda.synchronize()
        times[label] = e0.elapsed_time(e1)
    c = cs.cpu().numpy().astype(np.uint32)
    solved = c != 0xFFFFFFFF
    region = np.bincount(c[solved] & 3, minlength=4) / solved.sum()
    steps = np.bincount((c[solved] >> 2) & 3, minlength=3) / solved.sum()
    n_paths = len(np.unique(c[solved]))
    print(json.dumps({"census": True, "n": int(P.numel()), "solved": int(solved.sum()),
                      "distinct_paths": n_paths,
                      "region_fraction_R1_R4": region.round(4).tolist(),
                      "steps_fraction_2_3_4": steps.round(5).tolist(),
                      "ms_as_generated": times["as_generated"],
                      "ms_sorted_by_path": times["sorted_by_path"],
                      "launch_order": ["as_generated", "sorted_by_path"]}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(quotes are independent, so a multi-GPU run would shard the batch by contiguous "
              "index ranges with no exchange)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2604_27210_amd as fv
    fv._native.load()
    torch.cuda.init()
    wl, P, S, K, T, r, q, flag = make_inputs(a.n, torch, fv)
    stream = torch.cuda.current_stream()
    if a.census:
        census(fv, torch, P, S, K, T, r, q, flag)
        return

    def step():
        return fv.implied_vol("bsm", P, S, K, T, r, flag=flag, q=q, solver=a.solver)

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

    roof = None
    if LBR_FLOP_PER_QUOTE and a.solver == "lbr":
        ach = LBR_FLOP_PER_QUOTE * a.n / avg_kernel_s / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "traffic": None}
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
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, P.cpu().numpy(), a.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
