"""Writes ``svi_calibration_500.json``: the oracle's result of the 500-chain
SVI calibration (Black-76 chains drawn with seed 5, 200 Adam steps at
lr 1e-2, beta = (0.9, 0.999), eps 1e-8), the calibration use case the paper
gives for a differentiable implied volatility (section 1).

Everything here calls only ``oracle/``: the binary128 Black-76 price of the
perturbed SVI vols, its exact-root implied volatility as the target, and the
numpy Adam replay of ``oracle/svi.py``.  Run from the repository root:

    python tests/golden/make_svi_calibration.py

(about two minutes on eight cores).  The full-size GPU calibration test
repeats the same replay and checks that it reproduces the stored figures.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "svi_calibration_500.json")
N_CHAINS, SEED, STEPS, LR = 500, 5, 200, 1e-2
CHECKPOINTS = (0, 1, 9, 19, 49, 99, 149, 199)


def raw_of(th):
    """(a, b, rho, m, s) -> raw (a, b~, rho~, m, s~): b = softplus(b~),
    rho = tanh(rho~), s = softplus(s~)."""
    out = np.array(th, dtype=np.float64)
    out[:, 1] = np.log(np.expm1(th[:, 1]))
    out[:, 2] = np.arctanh(th[:, 2])
    out[:, 4] = np.log(np.expm1(th[:, 4]))
    return out


def oracle_problem(n_chains=N_CHAINS, seed=SEED):
    """(calibration draw, maturity index per quote, oracle IV targets with
    NaN where the oracle finds no root)."""
    import oracle
    from oracle import svi
    from paper_2604_27210_amd import workloads as W
    c = W.svi_calibration(n_chains, seed=seed)
    ch = c.chains
    mat = ch.mat_of_quote()
    chain = ch.chain_of_mat()[mat]
    sig_true = svi.svi_vols(raw_of(c.theta_true), ch.k, mat, ch.T) * (1.0 + c.eps)
    P = oracle.price("black76", ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0, sig_true, ch.flag)
    target, st = oracle.implied_vol("black76", P, ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0,
                                    ch.flag)
    return c, mat, np.where(st == 0, target, np.nan)


def rmse_vol_points(raw, c, mat, target):
    from oracle import svi
    ok = np.isfinite(target)
    v = svi.svi_vols(raw, c.chains.k, mat, c.chains.T)
    return float(100.0 * np.sqrt(np.mean((v[ok] - target[ok]) ** 2)))


def main():
    from oracle import svi
    c, mat, target = oracle_problem()
    raw0 = raw_of(c.theta0)
    th, losses = svi.adam_replay(raw0, c.chains.k, mat, c.chains.T, target, STEPS, lr=LR)
    rec = {
        "source": "oracle/ (binary128 Black-76 price and exact-root IV targets; numpy Adam "
                  "replay of oracle/svi.py), written by tests/golden/make_svi_calibration.py",
        "workload": {"n_chains": N_CHAINS, "seed": SEED, "n_quotes": int(c.chains.n),
                     "n_maturities": int(c.chains.n_mat), "steps": STEPS, "lr": LR,
                     "beta1": 0.9, "beta2": 0.999, "eps": 1e-8},
        "n_targets": int(np.isfinite(target).sum()),
        "initial_rmse_vol_points": rmse_vol_points(raw0, c, mat, target),
        "final_rmse_vol_points": rmse_vol_points(th, c, mat, target),
        "loss_at_step": {str(k): float(losses[k]) for k in CHECKPOINTS},
        "final_theta_abs_sum": float(np.abs(th).sum()),
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
