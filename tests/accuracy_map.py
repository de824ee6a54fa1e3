"""Accuracy of the GPU solvers and of the normalised Black evaluator over a
dense (x, s) plane, against the oracle (the paper's "worst-case relative
error on a dense grid of moneyness x total variance" figure, section 4).

The plane is reached through the Black-76 entry point with F = 1,
K = e^{-x} (x = ln(F/K) <= 0, out-of-the-money calls), T = 1, r = 0, so the
total volatility s is sigma itself and the price is sqrt(K) b(x, s).  Cells
whose price is not a positive binary64 number strictly inside its bounds are
left out.  For each cell block the table reports the largest relative error
in units of u = 2^-53:
  * b: fv_normalised_black against the oracle's binary128 b (rounded);
  * LBR / Halley: the GPU implied volatility against the oracle's exact root
    of the binary64 price, and the largest ratio error / parity tolerance.

Run as a script (GPU required) to print the markdown table:
    python tests/accuracy_map.py > accuracy_map.md
The GPU test test_gpu_accuracy_map.py runs a coarser plane and asserts the
bounds.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from _helpers import cond_abs, iv_tolerance  # noqa: E402

U = 2.0 ** -53


def plane(nx: int, ns: int):
    """x in {0} U -logspace(-4, log10(20)); s logspace(-3, log10(8))."""
    xs = np.concatenate([[0.0], -np.logspace(-4, np.log10(20.0), nx - 1)])
    ss = np.logspace(-3, np.log10(8.0), ns)
    X, S = np.meshgrid(xs, ss, indexing="ij")
    return xs, ss, X.ravel(), S.ravel()


def measure(fv, torch, nx=160, ns=160):
    xs, ss, x, s = plane(nx, ns)
    n = x.size
    K = np.exp(-x)
    one, zero = np.ones(n), np.zeros(n)
    calls = np.ones(n, dtype=np.int8)
    P = oracle.price("black76", one, K, one, zero, 0.0, s, calls)
    so, st = oracle.implied_vol("black76", P, one, K, one, zero, 0.0, calls)
    ok = (st == 0) & (P > 0)
    d = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    res = {}
    bo = oracle.normalised_black(x, s, 1)
    bg = fv.normalised_black(d(x), d(s)).cpu().numpy()
    with np.errstate(divide="ignore", invalid="ignore"):
        res["b"] = np.where(bo > 0, np.abs(bg - bo) / bo / U, np.nan)
    idx = np.where(ok)[0]
    tol = np.full(n, np.nan)
    tol_h = np.full(n, np.nan)
    ca = cond_abs("black76", P[idx], one[idx], K[idx], one[idx], zero[idx], 0.0, calls[idx])
    tol[idx] = iv_tolerance("lbr", so[idx], ca)
    tol_h[idx] = iv_tolerance("halley", so[idx], ca)
    # a tolerance that is not finite would accept any value
    res["inf_tol"] = int(np.sum(~np.isfinite(tol[idx])) + np.sum(~np.isfinite(tol_h[idx])))
    res["subnormal_price_cells"] = int(np.sum(P[idx] < 2.2250738585072014e-308))
    for solver, tl in (("lbr", tol), ("halley", tol_h)):
        sg, sst = fv.implied_vol("black76", d(P[idx]), d(one[idx]), d(K[idx]), d(one[idx]),
                                 d(zero[idx]), flag=d(calls[idx], torch.int8), solver=solver)
        sg, sst = sg.cpu().numpy(), sst.cpu().numpy()
        e = np.full(n, np.nan)
        r = np.full(n, np.nan)
        good = sst == 0
        e[idx[good]] = np.abs(sg[good] - so[idx][good]) / so[idx][good] / U
        r[idx[good]] = np.abs(sg[good] - so[idx][good]) / tl[idx][good]
        bad_status = idx[~good]
        res[solver] = e
        res[solver + "_ratio"] = r
        res[solver + "_status_mismatch"] = bad_status
    return xs, ss, res, ok


def blocks(v, nx, ns, bx, bs):
    """Max over (bx x bs) cell blocks of a field on the (nx, ns) plane."""
    a = v.reshape(nx, ns)
    out = np.full((bx, bs), np.nan)
    ex = np.linspace(0, nx, bx + 1).astype(int)
    es = np.linspace(0, ns, bs + 1).astype(int)
    for i in range(bx):
        for j in range(bs):
            blk = a[ex[i]:ex[i + 1], es[j]:es[j + 1]]
            if np.any(np.isfinite(blk)):
                out[i, j] = np.nanmax(blk)
    return out, ex, es


def main():
    import torch
    import paper_2604_27210_amd as fv
    fv._native.load()
    nx = ns = 160
    xs, ss, res, ok = measure(fv, torch, nx, ns)
    bx = bs = 10
    print("# Accuracy over the (x, s) plane -- %d x %d grid, %d cells with a solvable price\n"
          % (nx, ns, int(ok.sum())))
    print("Command: `python tests/accuracy_map.py` (GPU; the oracle is the reference).\n")
    print("x = ln(F/K) <= 0 (out-of-the-money calls via Black-76 with F = 1, T = 1, r = 0), "
          "s = sigma sqrt(T). Entries: the largest relative error in each block, in units of "
          "u = 2^-53 ('-': no solvable cell).\n")
    for key, title in (("b", "normalised Black b(x, s) (fv_normalised_black)"),
                       ("lbr", "LBR implied volatility"), ("halley", "Halley implied volatility")):
        t, ex, es = blocks(res[key], nx, ns, bx, bs)
        print("## %s\n" % title)
        print("| x \\ s | " + " | ".join("%.3g..%.3g" % (ss[es[j]], ss[es[j + 1] - 1])
                                       for j in range(bs)) + " |")
        print("|---" * (bs + 1) + "|")
        for i in range(bx):
            print("| %.3g..%.3g | " % (xs[ex[i]], xs[ex[i + 1] - 1]) +
                  " | ".join("-" if not np.isfinite(v) else "%.3g" % v for v in t[i]) + " |")
        allv = res[key][np.isfinite(res[key])]
        print("\nmax %.4g u, median %.3g u over %d cells" % (allv.max(), np.median(allv), allv.size))
        if key == "b":
            print("; solvable cells with a price below the normal binary64 range: %d; "
                  "cells with a non-finite parity tolerance: %d"
                  % (res["subnormal_price_cells"], res["inf_tol"]))
        if key != "b":
            rr = res[key + "_ratio"]
            rr = rr[np.isfinite(rr)]
            print("; largest error / parity tolerance %.3g; status mismatches %d\n"
                  % (rr.max(), len(res[key + "_status_mismatch"])))
        else:
            print()


if __name__ == "__main__":
    main()
