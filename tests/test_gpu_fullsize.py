"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (the library's default shapes), on sampled outputs that the
oracle computes one by one, plus properties checked on every output.

  * 10,000,000 wide-wing BSM quotes with 1% injected degenerate prices (both
    solvers): 20,000 random quotes, the last 777 (the ragged tail of the
    grid) and 3,000 injected quotes against the oracle; over all quotes, the
    status conventions, every injected quote flagged, every clean quote
    solved.
  * 2,000 ragged Black-76 chains (about 8.4M quotes) in one launch, both
    solvers: a sample against the oracle, and every quote solved.
  * The binary32 Halley path on the 10M batch rounded to float32, sampled.
  * The 1M differentiation workload's forward with the Greeks fused in:
    sampled Greeks against the oracle's.
  * The 1,000,000-quote differentiation workload through autograd: sampled
    gradients against the oracle's implicit-function gradient.
  * SVI calibration on 500 chains (2.08M quotes): the first 20 losses and
    the parameters after them against the oracle's Adam replay, then the
    benchmark's 200 graph-replayed steps (loss falls below 5% of its start,
    RMSE under 3 vol points).

Input prices always come from the oracle (binary128 pricing of the seeded
draws), never from the library."""
import numpy as np
import pytest

import oracle
from oracle import svi
from paper_2604_27210_amd import workloads as W

from _helpers import (GRAD_NAMES, GREEK_NAMES, assemble_prices, boundary_ambiguous, compare_iv,
                      grad_bad, greeks_bad)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_27210_amd as fv
    fv._native.load()
    return fv


def dev(a, dtype=torch.float64, grad=False):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)
    return t.requires_grad_(grad)


def _sample(n, rng, k=20_000, tail=777, extra=None):
    parts = [rng.choice(n, size=min(k, n), replace=False), np.arange(max(0, n - tail), n)]
    if extra is not None:
        parts.append(extra)
    return np.unique(np.concatenate(parts))


@pytest.fixture(scope="module")
def wide10m():
    wl = W.bsm_wide(10_000_000, seed=2)
    return wl, assemble_prices(wl)


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_wide_bsm_10m_sampled(fv, wide10m, solver):
    wl, P = wide10m
    n = wl.n
    sig, st = fv.implied_vol("bsm", dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r),
                             flag=dev(wl.flag, torch.int8), q=dev(wl.q), solver=solver)
    torch.cuda.synchronize()
    sig, st = sig.cpu().numpy(), st.cpu().numpy()
    assert sig.shape == (n,) and st.shape == (n,)
    inj = wl.kind != W.KIND_CLEAN
    rng = np.random.default_rng(11)
    idx = _sample(n, rng, extra=rng.choice(np.where(inj)[0], 3000, replace=False))
    res = compare_iv("bsm", solver, P[idx], wl.fs[idx], wl.K[idx], wl.T[idx], wl.r[idx],
                     wl.q[idx], wl.flag[idx], sig[idx], st[idx])
    assert res["n_ok"] > 0.99 * (~inj[idx]).sum()
    assert len(res["status_bad"]) == 0, res["status_bad"][:5]
    assert len(res["value_bad"]) == 0, (res["value_bad"][:5], res["max_ratio"])
    assert len(res["nan_bad"]) == 0
    # properties over all 10M outputs
    ok = st == 0
    assert np.all(np.isfinite(sig[ok]) & (sig[ok] > 0.0))
    assert np.all(np.isnan(sig[(st >= 2) & (st <= 4)]))
    assert np.all(sig[st == 1] == 0.0)
    assert not np.any(st == 4)  # every input is valid
    amb = boundary_ambiguous("bsm", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    assert np.all((st[inj] != 0) | amb[inj])
    clean = ~inj & ~amb
    # clean prices are solvable except where the binary64 price has rounded
    # onto a bound (the oracle flags those too; the sample above checks the
    # agreement quote by quote)
    assert (st[clean] == 0).mean() > 0.9999


def test_ragged_chains_full_sampled(fv):
    ch = W.b76_chains(2000, seed=3)
    flat = ch.flatten()
    P = oracle.price("black76", flat.fs, flat.K, flat.T, flat.r, 0.0, flat.sigma_true, flat.flag)
    sig, st = fv.implied_vol_chains(dev(ch.chain_mat_off, torch.int64),
                                    dev(ch.mat_quote_off, torch.int64), dev(ch.F), dev(ch.r),
                                    dev(ch.T), dev(P), dev(ch.K), dev(ch.flag, torch.int8))
    torch.cuda.synchronize()
    sig, st = sig.cpu().numpy(), st.cpu().numpy()
    assert sig.shape == (flat.n,)
    idx = _sample(flat.n, np.random.default_rng(12))
    res = compare_iv("black76", "lbr", P[idx], flat.fs[idx], flat.K[idx], flat.T[idx],
                     flat.r[idx], 0.0, flat.flag[idx], sig[idx], st[idx])
    assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0 and len(res["nan_bad"]) == 0
    assert res["n_ok"] > 0.99 * len(idx)
    # every quote of the chains is an out-of-the-money quote of a smile
    # price: solved everywhere
    assert (st == 0).mean() > 0.9999
    assert np.all(np.isfinite(sig[st == 0]))


def test_ragged_chains_full_halley_sampled(fv):
    ch = W.b76_chains(2000, seed=3)
    flat = ch.flatten()
    P = oracle.price("black76", flat.fs, flat.K, flat.T, flat.r, 0.0, flat.sigma_true, flat.flag)
    sig, st = fv.implied_vol_chains(dev(ch.chain_mat_off, torch.int64),
                                    dev(ch.mat_quote_off, torch.int64), dev(ch.F), dev(ch.r),
                                    dev(ch.T), dev(P), dev(ch.K), dev(ch.flag, torch.int8),
                                    solver="halley")
    torch.cuda.synchronize()
    sig, st = sig.cpu().numpy(), st.cpu().numpy()
    idx = _sample(flat.n, np.random.default_rng(14))
    res = compare_iv("black76", "halley", P[idx], flat.fs[idx], flat.K[idx], flat.T[idx],
                     flat.r[idx], 0.0, flat.flag[idx], sig[idx], st[idx])
    assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0 and len(res["nan_bad"]) == 0
    assert (st == 0).mean() > 0.9999


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_fused_greeks_1m_sampled(fv, solver):
    """The differentiation workload's forward with the Greeks fused in, at
    its full size: sampled Greeks, element by element, against the oracle's
    binary128 Greeks at the solved sigma (within 64 u kappa), and the sampled
    sigma against the oracle's root; NaN Greeks wherever the status is not
    OK (checked over every output)."""
    wl = W.bsm_diff(1_000_000, seed=4)
    P = assemble_prices(wl)
    sig, st, gk = fv.implied_vol("bsm", dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r),
                                 flag=dev(wl.flag, torch.int8), q=dev(wl.q), greeks=True,
                                 solver=solver)
    torch.cuda.synchronize()
    sig, st = sig.cpu().numpy(), st.cpu().numpy()
    gh = {k: v.cpu().numpy() for k, v in gk.items()}
    for k in gh:
        assert np.all(np.isnan(gh[k][st != 0])), k
    idx = _sample(wl.n, np.random.default_rng(15))
    res = compare_iv("bsm", solver, P[idx], wl.fs[idx], wl.K[idx], wl.T[idx], wl.r[idx],
                     wl.q[idx], wl.flag[idx], sig[idx], st[idx])
    assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
    idx = idx[st[idx] == 0]
    bad, worst = greeks_bad("bsm", wl.fs[idx], wl.K[idx], wl.T[idx], wl.r[idx], wl.q[idx],
                            sig[idx], wl.flag[idx], {k: v[idx] for k, v in gh.items()})
    print("fused-greeks-1m/%s: %d quotes, max err/tol %.3g" % (solver, len(idx), worst))
    for name in GREEK_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])


def test_binary32_10m_sampled(fv, wide10m):
    """The binary32 Halley path on the 10M wide workload rounded to float32,
    sampled against the oracle on the same binary32 inputs."""
    from test_gpu_f32 import compare_f32
    wl, P = wide10m
    A = [np.ascontiguousarray(x, dtype=np.float32) for x in (P, wl.fs, wl.K, wl.T, wl.r, wl.q)]
    t32 = [torch.from_numpy(a).to("cuda") for a in A]
    sig, st = fv.implied_vol_f32("bsm", *t32[:5], flag=dev(wl.flag, torch.int8), q=t32[5])
    torch.cuda.synchronize()
    sig, st = sig.cpu().numpy().astype(np.float64), st.cpu().numpy()
    inj = wl.kind != W.KIND_CLEAN
    rng = np.random.default_rng(16)
    idx = _sample(wl.n, rng, extra=rng.choice(np.where(inj)[0], 3000, replace=False))
    n_ok, worst = compare_f32("bsm", [a[idx].astype(np.float64) for a in A], wl.flag[idx],
                              sig[idx], st[idx])
    # float32 rounding puts more deep in-the-money prices onto their bounds
    # and leaves normalised prices below 2^-100 to the binary64 path (both
    # checked quote by quote above); about 91% of the clean sample is solved
    assert n_ok > 0.85 * (~inj[idx]).sum() and worst <= 1.0


def test_differentiation_1m_sampled(fv):
    wl = W.bsm_diff(1_000_000, seed=4)
    P = assemble_prices(wl)
    ins = [dev(P, grad=True), dev(wl.fs, grad=True), dev(wl.K, grad=True), dev(wl.T, grad=True),
           dev(wl.r, grad=True), dev(wl.q, grad=True)]
    sig, st = fv.implied_vol_autograd("bsm", ins[0], ins[1], ins[2], ins[3], ins[4],
                                      flag=dev(wl.flag, torch.int8), q=ins[5])
    w = dev(wl.extra["w"])
    (w * sig).sum().backward()
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    grads = np.stack([t.grad.cpu().numpy() for t in ins], 1)
    assert (st == 0).mean() > 0.999
    idx = _sample(wl.n, np.random.default_rng(13))
    sg = sig.detach().cpu().numpy()
    res = compare_iv("bsm", "lbr", P[idx], wl.fs[idx], wl.K[idx], wl.T[idx], wl.r[idx],
                     wl.q[idx], wl.flag[idx], sg[idx], st[idx])
    assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
    idx = idx[st[idx] == 0]
    # every sampled gradient element against the oracle's binary128 gradient
    # formula at the solved sigma
    bad, worst, nonfin = grad_bad("bsm", wl.fs[idx], wl.K[idx], wl.T[idx], wl.r[idx], wl.q[idx],
                                  sg[idx], wl.flag[idx], grads[idx], w=wl.extra["w"][idx],
                                  P=P[idx])
    print("autograd-1m: %d quotes, max err/tol %.3g" % (len(idx), worst))
    assert nonfin == 0
    for name in GRAD_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])
    # quotes that are not solved carry no gradient
    assert np.all(grads[st != 0] == 0.0)


def _raw(th):
    out = th.copy()
    out[:, 1] = np.log(np.expm1(th[:, 1]))
    out[:, 2] = np.arctanh(th[:, 2])
    out[:, 4] = np.log(np.expm1(th[:, 4]))
    return out


def test_calibration_500_chains_full(fv):
    """The 500-chain calibration as benchmarked (200 graph-replayed Adam
    steps) against the oracle's numpy replay of all 200 steps on the
    oracle's own targets: every loss, every parameter and the final RMSE;
    the replay also reproduces the stored figures of
    tests/golden/svi_calibration_500.json that the bench prints."""
    import json
    import os
    from paper_2604_27210_amd.calibrate import SviCalibrator, calibrate_svi, raw_from_natural
    c = W.svi_calibration(500, seed=5)
    ch = c.chains
    mat = ch.mat_of_quote()
    chain = ch.chain_of_mat()[mat]
    sig_true = svi.svi_vols(_raw(c.theta_true), ch.k, mat, ch.T) * (1.0 + c.eps)
    P = oracle.price("black76", ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0, sig_true, ch.flag)
    target, st = oracle.implied_vol("black76", P, ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0,
                                    ch.flag)
    target = np.where(st == 0, target, np.nan)
    cal = SviCalibrator(dev(ch.chain_mat_off, torch.int64), dev(ch.mat_quote_off, torch.int64),
                        dev(ch.F), dev(ch.r), dev(ch.T), dev(ch.K), dev(ch.flag, torch.int8),
                        dev(target), raw_from_natural(c.theta0), lr=1e-2)
    calibrate_svi(cal, 200, graph=True)
    torch.cuda.synchronize()
    L = cal.losses()
    th = cal.theta.cpu().numpy().reshape(-1, 5)
    ok = np.isfinite(target)
    rmse = 100 * np.sqrt(np.mean((cal.vols().cpu().numpy()[ok] - target[ok]) ** 2))
    th_o, L_o = svi.adam_replay(_raw(c.theta0), ch.k, mat, ch.T, target, 200)
    rmse_o = 100 * np.sqrt(np.mean((svi.svi_vols(th_o, ch.k, mat, ch.T)[ok] - target[ok]) ** 2))
    print("calibration-500: %d quotes, %d maturities; rmse gpu %.12f oracle %.12f; "
          "max loss rel dev %.3g; max theta dev %.3g"
          % (ch.n, ch.n_mat, rmse, rmse_o, np.max(np.abs(L / L_o - 1)), np.max(np.abs(th - th_o))))
    assert len(L) == 200 and np.all(np.isfinite(L))
    np.testing.assert_allclose(L[:20], L_o[:20], rtol=1e-9)
    np.testing.assert_allclose(L, L_o, rtol=1e-6)
    np.testing.assert_allclose(th, th_o, rtol=1e-6, atol=1e-9)
    assert abs(rmse - rmse_o) <= 1e-6
    assert L[-1] < 0.05 * L[0]
    with open(os.path.join(os.path.dirname(__file__), "golden", "svi_calibration_500.json")) as fh:
        gold = json.load(fh)
    assert gold["workload"]["n_quotes"] == ch.n and gold["workload"]["steps"] == 200
    assert abs(gold["final_rmse_vol_points"] - rmse_o) <= 1e-9 * rmse_o
    for k, v in gold["loss_at_step"].items():
        assert abs(v - L_o[int(k)]) <= 1e-9 * v, k
