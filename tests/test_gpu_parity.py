"""GPU parity: the HIP library against the binary128 oracle, element by
element, through the C ABI (via the thin Python binding)."""
import numpy as np
import pytest

import oracle
from paper_2604_27210_amd import workloads as W

from _helpers import (GRAD_NAMES, GREEK_NAMES, U, assemble_prices, boundary_ambiguous,
                      compare_iv, cond_abs, forward_discount, grad_bad, greek_terms, greeks_bad)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_27210_amd as fv
    fv._native.load()
    return fv


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.cpu().numpy()


def run_iv(fv, wl, P, solver, greeks=False):
    q = dev(wl.q) if wl.model == "bsm" else None
    out = fv.implied_vol(wl.model, dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r),
                         flag=dev(wl.flag, torch.int8), q=q, solver=solver, greeks=greeks)
    torch.cuda.synchronize()
    return out


def _report(name, res):
    print("%s: ok=%d status_bad=%d value_bad=%d (non-finite tolerance %d) nan_bad=%d "
          "ambiguous=%d not compared by value=%d max err/tol=%.3f" % (
              name, res["n_ok"], len(res["status_bad"]), len(res["value_bad"]), res["inf_tol"],
              len(res["nan_bad"]), res["ambiguous"], res["excluded"], res["max_ratio"]), flush=True)


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_bs_small_batch(fv, solver):
    """Black-Scholes, 4,096 quotes (the small seeded workload), both solvers."""
    wl = W.bs_small()
    P = assemble_prices(wl)
    sig, st = run_iv(fv, wl, P, solver)
    res = compare_iv(wl.model, solver, P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag, host(sig),
                     host(st))
    _report("bs_small/" + solver, res)
    assert len(res["status_bad"]) == 0
    assert len(res["value_bad"]) == 0
    assert len(res["nan_bad"]) == 0
    assert res["n_ok"] > 3900


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_bsm_wide_sample(fv, solver):
    """Black-Scholes-Merton wide wings with 1% injected degenerate prices,
    200,003 quotes (several thousand workgroups and a ragged tail)."""
    wl = W.bsm_wide(200_003, seed=2)
    P = assemble_prices(wl)
    sig, st = run_iv(fv, wl, P, solver)
    res = compare_iv(wl.model, solver, P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag, host(sig),
                     host(st))
    _report("bsm_wide/" + solver, res)
    assert len(res["status_bad"]) == 0
    assert len(res["value_bad"]) == 0
    assert len(res["nan_bad"]) == 0
    st_h = host(st)
    # every injected quote is flagged, none silently solved
    inj = wl.kind != W.KIND_CLEAN
    amb = boundary_ambiguous(wl.model, P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    assert np.all((st_h[inj] != 0) | amb[inj])


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_models_and_flags(fv, model):
    rng = np.random.default_rng(7)
    n = 20_000
    S = rng.uniform(20, 300, n)
    T = np.exp(rng.uniform(np.log(1 / 365), np.log(5), n))
    r = rng.uniform(-0.01, 0.08, n)
    q = rng.uniform(0, 0.05, n) if model == "bsm" else np.zeros(n)
    sig = np.exp(rng.uniform(np.log(0.02), np.log(2.5), n))
    z = rng.uniform(-5, 5, n)
    F, _ = forward_discount(model, S, T, r, q)
    K = F * np.exp(-z * sig * np.sqrt(T))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    wl = W.Flat(model, S, K, T, r, q, sig, flag)
    P = assemble_prices(wl)
    for solver in ("lbr", "halley"):
        s, st = run_iv(fv, wl, P, solver)
        res = compare_iv(model, solver, P, S, K, T, r, q, flag, host(s), host(st))
        _report("%s/%s" % (model, solver), res)
        assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
        assert len(res["nan_bad"]) == 0


def test_edge_cases(fv):
    """Empty batch, single quote, at-the-money exactly, broadcast scalars,
    invalid inputs, degenerate prices, extreme wings, huge and tiny vols."""
    # n == 0 is a no-op
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    s0, st0 = fv.implied_vol("bsm", e, e, e, e, e, flag="c", q=e)
    assert s0.numel() == 0
    # exactly at the money (F == K) for Black-76, both flags, broadcast F/T/r
    K = np.array([100.0, 100.0, 100.0, 100.0])
    sig = np.array([0.01, 0.3, 1.5, 4.0])
    T, r = 0.75, 0.02
    for fl in (1, -1):
        P = oracle.price("black76", 100.0, K, T, r, 0.0, sig, fl)
        s, st = fv.implied_vol("black76", dev(P), 100.0, dev(K), T, r, flag=fl)
        s, st = host(s), host(st)
        assert np.all(st == 0)
        np.testing.assert_allclose(s, sig, rtol=1e-12)
    # invalid inputs and degenerate prices
    P = np.array([np.nan, 5.0, 5.0, 5.0, 5.0, -1.0, 1e9, 0.0])
    S = np.array([100.0, -1.0, 100.0, 100.0, 100.0, 100.0, 100.0, 100.0])
    Kx = np.array([100.0, 100.0, 0.0, 100.0, 100.0, 100.0, 100.0, 150.0])
    Tx = np.array([1.0, 1.0, 1.0, 0.0, np.inf, 1.0, 1.0, 1.0])
    s, st = fv.implied_vol("bs", dev(P), dev(S), dev(Kx), dev(Tx), 0.01, flag="c")
    s, st = host(s), host(st)
    assert list(st) == [4, 4, 4, 4, 4, 2, 3, 1]
    assert np.all(np.isnan(s[:7])) and s[7] == 0.0
    # extreme wings and vol levels against the oracle
    rng = np.random.default_rng(3)
    n = 5000
    h = -np.exp(rng.uniform(np.log(1e-4), np.log(30), n))
    t = np.exp(rng.uniform(np.log(1e-4), np.log(5), n))
    x = 2 * h * t
    F = 100.0
    Kw = F * np.exp(-x)
    Tw = rng.uniform(0.01, 3, n)
    sw = 2 * t / np.sqrt(Tw)
    fl = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    wl = W.Flat("black76", np.full(n, F), Kw, Tw, np.zeros(n), np.zeros(n), sw, fl)
    P = assemble_prices(wl)
    for solver in ("lbr", "halley"):
        s, st = run_iv(fv, wl, P, solver)
        res = compare_iv("black76", solver, P, wl.fs, Kw, Tw, 0.0 * Tw, 0.0 * Tw, fl, host(s),
                         host(st))
        _report("wings/" + solver, res)
        assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0


def test_ragged_sizes_and_launch_shapes(fv):
    """Sizes around wave and workgroup multiples under every launch shape give
    bitwise the same per-quote results as the default shape (the per-quote
    code does not depend on the shape), and the default agrees with the
    oracle."""
    wl_all = W.bsm_wide(70_000, seed=12, inject=0.01)
    P_all = assemble_prices(wl_all)
    ref = {}
    for solver in ("lbr", "halley"):
        s, st = run_iv(fv, wl_all, P_all, solver)
        ref[solver] = (torch.nan_to_num(s, nan=-7.0), st)
        res = compare_iv("bsm", solver, P_all, wl_all.fs, wl_all.K, wl_all.T, wl_all.r,
                         wl_all.q, wl_all.flag, host(s), host(st))
        assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
    saved = {k: fv.get_launch(k) for k in ("iv_lbr", "iv_halley")}
    try:
        for block, qpt in ((64, 1), (128, 2), (256, 4), (512, 3), (64, 16)):
            fv.set_launch("iv_lbr", block, qpt)
            fv.set_launch("iv_halley", block, qpt)
            for n in sorted({1, 63, 64, 65, 257, block * qpt - 1, block * qpt + 1, 70_000}):
                idx = np.arange(n)
                wl = wl_all.take(idx)
                for solver in ("lbr", "halley"):
                    s, st = run_iv(fv, wl, P_all[idx], solver)
                    rs, rst = ref[solver]
                    assert torch.equal(torch.nan_to_num(s, nan=-7.0), rs[:n]), (block, qpt, n, solver)
                    assert torch.equal(st, rst[:n]), (block, qpt, n, solver)
    finally:
        for k, (b, q) in saved.items():
            fv.set_launch(k, b, q)
    # bad shapes are rejected
    from paper_2604_27210_amd._native import FastvolError
    with pytest.raises(FastvolError):
        fv.set_launch("iv_lbr", 96, 1)
    with pytest.raises(FastvolError):
        fv.set_launch("iv_lbr", 1024, 1)


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_price_and_greeks(fv, model):
    rng = np.random.default_rng(17)
    n = 30_000
    S = rng.uniform(20, 300, n)
    T = np.exp(rng.uniform(np.log(1 / 365), np.log(5), n))
    r = rng.uniform(-0.01, 0.08, n)
    q = rng.uniform(0, 0.05, n) if model == "bsm" else np.zeros(n)
    sig = np.exp(rng.uniform(np.log(0.02), np.log(2.5), n))
    z = rng.uniform(-6, 6, n)
    F, D = forward_discount(model, S, T, r, q)
    K = F * np.exp(-z * sig * np.sqrt(T))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    qd = dev(q) if model == "bsm" else None
    p = host(fv.price(model, dev(S), dev(K), dev(T), dev(r), dev(sig), flag=dev(flag, torch.int8),
                      q=qd))
    po = oracle.price(model, S, K, T, r, q, sig, flag)
    # first-order condition number of the price in its inputs (relative units)
    g = oracle.greeks(model, S, K, T, r, q, sig, flag)
    dPdK = -flag * D * _ncdf(flag * (np.log(F / K) / (sig * np.sqrt(T)) - 0.5 * sig * np.sqrt(T)))
    cond = (np.abs(g["delta"] * S) + np.abs(dPdK * K) + np.abs(g["theta"] * T) +
            np.abs(g["vega"] * sig) + np.abs(g["rho"] * r) + np.abs(S * T * q * D * F / S))
    tol = 16 * U * (np.abs(po) + cond)
    bad = ~(np.abs(p - po) <= tol)
    assert bad.sum() == 0, (np.where(bad)[0][:5], p[bad][:5], po[bad][:5])
    gd = fv.greeks(model, dev(S), dev(K), dev(T), dev(r), dev(sig), flag=dev(flag, torch.int8), q=qd)
    bad, worst = greeks_bad(model, S, K, T, r, q, sig, flag, {k: host(v) for k, v in gd.items()},
                            ref=g, P=po)
    print("greeks/%s: max err/tol %.3g" % (model, worst))
    for name in GREEK_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])


def _ncdf(x):
    from scipy.special import ndtr
    return ndtr(x)


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_fused_greeks_match_separate_call_and_oracle(fv, solver):
    """The Greeks fused into the solve, element by element: against the
    oracle's binary128 Greeks at the solved sigma (within 64 u kappa), and
    against fv_greeks at that sigma (Black-Scholes-Merton's Greeks do not use
    the price, so both launches evaluate the same expressions, but each
    kernel's compiler contracts d1 = ln(F/K)/s + s/2 and theta's three-term
    sum into fused multiply-adds on its own): within 8 u kappa of the value
    (of theta's terms for theta).  NaN wherever the status is not OK."""
    wl = W.bsm_diff(50_000, seed=4)
    P = assemble_prices(wl)
    sig, st, gk = run_iv(fv, wl, P, solver, greeks=True)
    g2 = fv.greeks("bsm", dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r), sig,
                   flag=dev(wl.flag, torch.int8), q=dev(wl.q))
    st, sg = host(st), host(sig)
    ok = st == 0
    assert ok.mean() > 0.999
    i = np.where(ok)[0]
    kappa, theta_terms = greek_terms("bsm", wl.fs[i], wl.K[i], wl.T[i], wl.r[i], wl.q[i], sg[i],
                                     wl.flag[i], P[i])
    for name in gk:
        a = host(gk[name])
        assert np.all(np.isnan(a[~ok])), name
        b = host(g2[name])
        scale = theta_terms if name == "theta" else np.abs(b[i])
        assert np.all(np.abs(a[i] - b[i]) <= 8 * U * kappa * scale), name
    bad, worst = greeks_bad("bsm", wl.fs[i], wl.K[i], wl.T[i], wl.r[i], wl.q[i], sg[i],
                            wl.flag[i], {k: host(v)[i] for k, v in gk.items()})
    print("fused-greeks/%s: max err/tol %.3g" % (solver, worst))
    for name in GREEK_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])


def test_backward_matches_oracle_gradient(fv):
    wl = W.bsm_diff(100_000, seed=4)
    P = assemble_prices(wl)
    sig, st = run_iv(fv, wl, P, "lbr")
    w = dev(wl.extra["w"])
    gr = fv.implied_vol_backward("bsm", dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r), sig,
                                 w, flag=dev(wl.flag, torch.int8), q=dev(wl.q))
    st, sg = host(st), host(sig)
    ok = st == 0
    assert ok.mean() > 0.999
    wh = wl.extra["w"]
    got = np.stack([host(gr[name]) for name in GRAD_NAMES], 1)
    # unsolved quotes carry no gradient
    assert np.all(got[~ok] == 0.0)
    # every solved quote: the gradient formula at the solved sigma, against
    # the oracle's binary128 formula at the same sigma
    i = np.where(ok)[0]
    bad, worst, nonfin = grad_bad("bsm", wl.fs[i], wl.K[i], wl.T[i], wl.r[i], wl.q[i], sg[i],
                                  wl.flag[i], got[i], w=wh[i], P=P[i])
    print("backward: max err/tol %.3g, non-finite reference values %d" % (worst, nonfin))
    assert nonfin == 0
    for name in GRAD_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])
    # and the solved sigma is the oracle's root, so this is also the
    # gradient at the root within the root's tolerance
    res = compare_iv("bsm", "lbr", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag, sg, st)
    assert len(res["value_bad"]) == 0 and len(res["status_bad"]) == 0


def test_chains_match_flat_and_oracle(fv):
    ch = W.b76_chains(60, seed=3)
    flat = ch.flatten()
    P = oracle.price("black76", flat.fs, flat.K, flat.T, flat.r, 0.0, flat.sigma_true, flat.flag)
    saved = fv.get_launch("chains")
    for solver in ("lbr", "halley"):
        for block, qpt in ((256, 1), (128, 4), (512, 2)):
            fv.set_launch("chains", block, qpt)
            sc, stc = fv.implied_vol_chains(
                dev(ch.chain_mat_off, torch.int64), dev(ch.mat_quote_off, torch.int64), dev(ch.F),
                dev(ch.r), dev(ch.T), dev(P), dev(ch.K), dev(ch.flag, torch.int8), solver=solver)
            sf, stf = fv.implied_vol("black76", dev(P), dev(flat.fs), dev(flat.K), dev(flat.T),
                                     dev(flat.r), flag=dev(flat.flag, torch.int8), solver=solver)
            torch.cuda.synchronize()
            if solver == "lbr":
                # same per-quote code path: bitwise identical to the flat kernel
                assert torch.equal(stc, stf)
                assert torch.equal(torch.nan_to_num(sc, nan=-1.0), torch.nan_to_num(sf, nan=-1.0))
            res = compare_iv("black76", solver, P, flat.fs, flat.K, flat.T, flat.r, 0.0 * flat.T,
                             flat.flag, host(sc), host(stc))
            assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
    fv.set_launch("chains", *saved)


def test_normalised_black_matches_oracle(fv):
    rng = np.random.default_rng(23)
    n = 100_000
    h = -np.exp(rng.uniform(np.log(1e-3), np.log(36), n))
    t = np.exp(rng.uniform(np.log(1e-5), np.log(6), n))
    x = 2 * h * t * np.where(rng.random(n) < 0.5, 1, -1)
    s = 2 * t
    fl = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    b = host(fv.normalised_black(dev(x), dev(s), dev(fl, torch.int8)))
    bo = oracle.normalised_black(x, s, fl)
    ok = bo > 1e-300
    # condition number of b in x (the kernel rounds h = x/s): |x db/dx| / b
    hh, tt = x / s, s / 2
    from scipy.special import ndtr
    bx = 0.5 * (np.exp(x / 2) * ndtr(fl * (hh + tt)) + np.exp(-x / 2) * ndtr(fl * (hh - tt)))
    cond = np.abs(x * bx) / np.maximum(bo, 1e-300)
    rel = np.abs(b - bo) / np.maximum(bo, 1e-300)
    bad = ok & ~(rel <= 64 * U * (1 + cond) + 1e-15)
    assert bad.sum() == 0, (np.where(bad)[0][:5], rel[bad][:5], cond[bad][:5])


def test_invalid_calls_raise(fv):
    d = dev(np.ones(4))
    from paper_2604_27210_amd._native import FastvolError
    with pytest.raises(FastvolError):
        fv.implied_vol(7, d, d, d, d, d)
    with pytest.raises(FastvolError):
        fv.implied_vol("bsm", d, d, d, d, d, solver=5)
    with pytest.raises((ValueError, TypeError)):
        fv.implied_vol("bsm", d, d, d.float(), d, d)


def test_autotune_per_size_class_and_tuning_file(fv, tmp_path):
    """fv_autotune keeps a valid shape per (family, model, size class), the
    launches of that class use it, per-quote results do not change, and a
    saved tuning file restores the table after a reset (and only on this
    architecture)."""
    wl = W.bsm_wide(50_000, seed=21, inject=0.0)
    P = assemble_prices(wl)
    s_ref, st_ref = run_iv(fv, wl, P, "lbr")
    kernels = ("price", "iv_lbr", "iv_halley", "greeks", "backward", "chains", "iv_halley_f32")
    saved = {k: fv.get_launch(k) for k in kernels}
    try:
        fv.reset_tuning()
        untuned = fv.launch_shape("iv_lbr", "bsm", 50_000)
        tuned = {}
        for n in (50_000, 1 << 20):
            b, q = fv.autotune("iv_lbr", "bsm", n)
            assert b % 64 == 0 and 64 <= b <= 512 and 1 <= q <= 8
            tuned[n] = (b, q)
            # every batch of the same size class launches with it
            assert fv.launch_shape("iv_lbr", "bsm", n) == (b, q)
        # another model's class is untouched
        assert fv.launch_shape("iv_lbr", "black76", 50_000) == untuned
        s, st = run_iv(fv, wl, P, "lbr")
        assert torch.equal(torch.nan_to_num(s, nan=-1.0), torch.nan_to_num(s_ref, nan=-1.0))
        assert torch.equal(st, st_ref)
        for kern in ("price", "iv_halley", "greeks", "backward", "chains", "iv_halley_f32"):
            b, q = fv.autotune(kern, "black76" if kern == "chains" else "bsm", 1 << 19)
            assert b % 64 == 0 and 1 <= q <= 8
        path = tmp_path / "tuning.json"
        fv.save_tuning(str(path))
        text = path.read_text()
        assert '"arch": "gfx950' in text
        fv.reset_tuning()
        assert fv.launch_shape("iv_lbr", "bsm", 50_000) == untuned
        fv.load_tuning(str(path))
        for n, bq in tuned.items():
            assert fv.launch_shape("iv_lbr", "bsm", n) == bq
        # a file written on another architecture is refused, nothing applied
        other = tmp_path / "other.json"
        other.write_text(text.replace('"arch": "gfx950', '"arch": "gfx000'))
        from paper_2604_27210_amd._native import FastvolError
        with pytest.raises(FastvolError):
            fv.load_tuning(str(other))
        for n, bq in tuned.items():
            assert fv.launch_shape("iv_lbr", "bsm", n) == bq
        # an explicit shape wins over the tuned classes of its family
        fv.set_launch("iv_lbr", 256, 1)
        assert fv.launch_shape("iv_lbr", "bsm", 1 << 20) == (256, 1)
    finally:
        fv.reset_tuning()
        for k, (b, q) in saved.items():
            fv.set_launch(k, b, q)


def test_scale_invariance(fv):
    """The implied volatility is homogeneous of degree 0 in (price, S, K):
    scaling all three by 2^k (even k, exact in binary64) must give bitwise
    the unscaled result, also where F K itself leaves the binary64 range
    (|k| >= 600); inputs below the normal range are invalid."""
    rng = np.random.default_rng(5)
    n = 4096
    S = np.full(n, 100.0)
    K = 100.0 * np.exp(rng.uniform(-0.5, 0.5, n))
    T = rng.uniform(0.1, 2.0, n)
    r = np.full(n, 0.03)
    q = np.full(n, 0.01)
    sig = rng.uniform(0.1, 0.6, n)
    fl = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int8)
    P = oracle.price("bsm", S, K, T, r, q, sig, fl)
    for solver in ("lbr", "halley"):
        ref = None
        for k in (0, 300, 600, 900, -300, -600):
            f = 2.0 ** k
            s, st = fv.implied_vol("bsm", dev(P * f), dev(S * f), dev(K * f), dev(T), dev(r),
                                   flag=dev(fl, torch.int8), q=dev(q), solver=solver)
            s, st = host(s), host(st)
            if ref is None:
                ref = (s, st)
                assert (st == 0).mean() > 0.97
            assert np.array_equal(st, ref[1]), (solver, k)
            assert np.array_equal(np.nan_to_num(s, nan=-1.0), np.nan_to_num(ref[0], nan=-1.0)), (solver, k)
    # S or K below the smallest normal binary64: invalid, not garbage
    s, st = fv.implied_vol("bs", dev(np.array([5.0, 5.0])), dev(np.array([1e-310, 100.0])),
                           dev(np.array([100.0, 1e-310])), 1.0, 0.0, flag="c")
    assert list(host(st)) == [4, 4] and np.all(np.isnan(host(s)))


def _fuzz_quotes(model, n=40_000):
    """Seeded quotes beyond the configured workloads: S over eight decades,
    sigma 1e-4..10, T 1e-6..50 years, r -0.1..0.3, q 0..0.3 (BSM), strikes
    at |z| <= 12 standard deviations, both flags."""
    rng = np.random.default_rng({"black76": 31, "bs": 32, "bsm": 33}[model])
    S = np.exp(rng.uniform(np.log(1e-3), np.log(1e5), n))
    T = np.exp(rng.uniform(np.log(1e-6), np.log(50.0), n))
    r = rng.uniform(-0.1, 0.3, n)
    q = rng.uniform(0.0, 0.3, n) if model == "bsm" else np.zeros(n)
    sig = np.exp(rng.uniform(np.log(1e-4), np.log(10.0), n))
    z = rng.uniform(-12, 12, n)
    F, D = forward_discount(model, S, T, r, q)
    K = F * np.exp(-z * sig * np.sqrt(T))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return rng, S, K, T, r, q, sig, flag


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_fuzz_extreme_ranges(fv, model):
    """The fuzz quotes' prices, plus 2% degenerate prices -- both solvers
    against the oracle."""
    rng, S, K, T, r, q, sig, flag = _fuzz_quotes(model)
    n = len(S)
    P = oracle.price(model, S, K, T, r, q, sig, flag)
    deg = rng.random(n) < 0.02
    P[deg] = P[deg] * rng.choice([0.0, -1.0, 1e6], deg.sum())
    for solver in ("lbr", "halley"):
        s, st = fv.implied_vol(model, dev(P), dev(S), dev(K), dev(T), dev(r),
                               flag=dev(flag, torch.int8), q=dev(q) if model == "bsm" else None,
                               solver=solver)
        res = compare_iv(model, solver, P, S, K, T, r, q, flag, host(s), host(st))
        _report("fuzz/%s/%s" % (model, solver), res)
        assert len(res["status_bad"]) == 0, res["status_bad"][:5]
        assert len(res["value_bad"]) == 0, (res["value_bad"][:5], res["max_ratio"])
        assert len(res["nan_bad"]) == 0


def _long_dated_quotes(model, n=40_000):
    """Long maturities with high rates (r T up to 40), negative q."""
    rng = np.random.default_rng({"black76": 61, "bs": 62, "bsm": 63}[model])
    S = np.exp(rng.uniform(np.log(1e-2), np.log(1e4), n))
    T = rng.uniform(20.0, 80.0, n)
    r = rng.uniform(-0.2, 0.5, n)
    q = rng.uniform(-0.1, 0.4, n) if model == "bsm" else np.zeros(n)
    sig = np.exp(rng.uniform(np.log(1e-2), np.log(1.0), n))
    z = rng.uniform(-6, 6, n)
    F, D = forward_discount(model, S, T, r, q)
    K = F * np.exp(-z * sig * np.sqrt(T))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return rng, S, K, T, r, q, sig, flag


@pytest.mark.parametrize("recipe", ["wide", "long_dated"])
@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_fuzz_greeks_and_gradient(fv, model, recipe):
    """Greeks and the implied-volatility gradient at the fuzz quotes' exact
    roots (the oracle's, rounded to binary64), against the oracle's binary128
    values, element by element (bounds: _helpers.greek_terms)."""
    _, S, K, T, r, q, sig, flag = (_fuzz_quotes if recipe == "wide" else _long_dated_quotes)(model)
    P = oracle.price(model, S, K, T, r, q, sig, flag)
    so, sto = oracle.implied_vol(model, P, S, K, T, r, q, flag)
    ok = (sto == 0) & (so > 0)
    S, K, T, r, q, flag, P, so = (a[ok] for a in (S, K, T, r, q, flag, P, so))
    qd = dev(q) if model == "bsm" else None
    fl = dev(flag, torch.int8)
    gd = fv.greeks(model, dev(S), dev(K), dev(T), dev(r), dev(so), flag=fl, q=qd)
    bad, worst = greeks_bad(model, S, K, T, r, q, so, flag, {k: host(v) for k, v in gd.items()})
    print("fuzz-greeks/%s/%s: max err/tol=%.3g" % (recipe, model, worst))
    for name in GREEK_NAMES:
        assert len(bad[name]) == 0, (model, name, bad[name][:5])
    w = np.random.default_rng(7).standard_normal(len(S))
    gr = fv.implied_vol_backward(model, dev(P), dev(S), dev(K), dev(T), dev(r), dev(so), dev(w),
                                 flag=fl, q=qd)
    got = np.stack([host(gr[name]) for name in GRAD_NAMES], 1)
    bad, worst, nonfin = grad_bad(model, S, K, T, r, q, so, flag, got, w=w, P=P)
    print("fuzz-grad/%s/%s: max err/tol=%.3g, %d reference values beyond binary64" % (
        recipe, model, worst, nonfin))
    for name in GRAD_NAMES:
        assert len(bad[name]) == 0, (model, name, bad[name][:5])
    # the gradient at the exact root is the root's gradient
    go = oracle.iv_grad(model, P, S, K, T, r, q, flag)
    go_at = oracle.iv_grad_at(model, S, K, T, r, q, so, flag)
    fin = np.isfinite(go) & (np.abs(go) < 1e300)
    assert np.all(np.abs(go_at[fin] - go[fin]) <= 1e-6 * np.abs(go[fin]) + 1e-300)


def test_chains_edge_structures(fv):
    """Ragged structures the configured chains never produce: chains with
    no maturities (also leading and trailing), maturities with no quotes,
    one quote, a wave and a wave plus one, and thousands; forwards over
    seven decades, T from 1e-5 to 30 years, r from -0.1 to 0.3, |z| <= 8.
    The chain kernel must equal the flat kernel bitwise (LBR) and both
    solvers must match the oracle."""
    rng = np.random.default_rng(41)
    n_chains = 200
    mpc = rng.choice([0, 1, 2, 5, 30], n_chains, p=[0.1, 0.3, 0.3, 0.2, 0.1])
    mpc[:3] = 0
    mpc[-3:] = 0
    n_mat = int(mpc.sum())
    qpm = rng.choice([0, 1, 3, 64, 65, 700, 5000], n_mat, p=[0.15, 0.2, 0.2, 0.15, 0.13, 0.15, 0.02])
    cmo = np.concatenate([[0], np.cumsum(mpc)]).astype(np.int64)
    mqo = np.concatenate([[0], np.cumsum(qpm)]).astype(np.int64)
    n = int(mqo[-1])
    F = np.exp(rng.uniform(np.log(1e-2), np.log(1e5), n_chains))
    r = rng.uniform(-0.1, 0.3, n_chains)
    T = np.exp(rng.uniform(np.log(1e-5), np.log(30.0), n_mat))
    chain_of_mat = np.repeat(np.arange(n_chains), mpc)
    mat_of_q = np.repeat(np.arange(n_mat), qpm)
    Fq, rq, Tq = F[chain_of_mat][mat_of_q], r[chain_of_mat][mat_of_q], T[mat_of_q]
    sig = np.exp(rng.uniform(np.log(1e-3), np.log(5.0), n))
    z = rng.uniform(-8, 8, n)
    K = Fq * np.exp(-z * sig * np.sqrt(Tq))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    P = oracle.price("black76", Fq, K, Tq, rq, 0.0, sig, flag)
    for solver in ("lbr", "halley"):
        sc, stc = fv.implied_vol_chains(dev(cmo, torch.int64), dev(mqo, torch.int64), dev(F), dev(r),
                                        dev(T), dev(P), dev(K), dev(flag, torch.int8), solver=solver)
        sf, stf = fv.implied_vol("black76", dev(P), dev(Fq), dev(K), dev(Tq), dev(rq),
                                 flag=dev(flag, torch.int8), solver=solver)
        torch.cuda.synchronize()
        if solver == "lbr":
            assert torch.equal(stc, stf)
            assert torch.equal(torch.nan_to_num(sc, nan=-1.0), torch.nan_to_num(sf, nan=-1.0))
        res = compare_iv("black76", solver, P, Fq, K, Tq, rq, 0.0 * Tq, flag, host(sc), host(stc))
        _report("chains-edge/%s (n=%d, %d maturities)" % (solver, n, n_mat), res)
        assert len(res["status_bad"]) == 0, res["status_bad"][:5]
        assert len(res["value_bad"]) == 0, (res["value_bad"][:5], res["max_ratio"])
        assert len(res["nan_bad"]) == 0


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_fuzz_long_dated_and_far_wings(fv, model):
    """Beyond the first fuzz: S over ten decades, T up to 80 years with r up
    to 0.5 (exponents r T of tens, where the forward and discount factor
    must carry the rounding of their exponents), negative q, sigma up to 20
    and |z| up to 15, plus quotes deep in the upper wing (|x| in [400, 650],
    s in [28, 50]), where iterates above the root meet b' and b_max - b
    below the normal range together.
    Both solvers against the oracle."""
    rng = np.random.default_rng({"black76": 51, "bs": 52, "bsm": 53}[model])
    n, m = 100_000, 4_000
    S = np.exp(rng.uniform(np.log(1e-4), np.log(1e6), n + m))
    T = np.exp(rng.uniform(np.log(1e-7), np.log(80.0), n + m))
    r = rng.uniform(-0.2, 0.5, n + m)
    q = rng.uniform(-0.1, 0.4, n + m) if model == "bsm" else np.zeros(n + m)
    sig = np.exp(rng.uniform(np.log(1e-5), np.log(20.0), n + m))
    z = rng.uniform(-15, 15, n + m)
    flag = np.where(rng.random(n + m) < 0.5, 1, -1).astype(np.int8)
    with np.errstate(over="ignore", invalid="ignore"):  # overflowing strikes are invalid quotes
        F, D = forward_discount(model, S, T, r, q)
        K = F * np.exp(-z * sig * np.sqrt(T))
    # the far upper wing: out-of-the-money |x| and total volatility s chosen
    # (calls K = F e^{|x|}, puts K = F e^{-|x|}; forwards kept so that K
    # stays finite)
    xw = rng.uniform(400.0, 650.0, m)
    sw = rng.uniform(28.0, 50.0, m)
    S[n:] = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), m))
    T[n:] = rng.uniform(0.5, 20.0, m)
    sig[n:] = sw / np.sqrt(T[n:])
    F, D = forward_discount(model, S, T, r, q)
    K[n:] = F[n:] * np.exp(flag[n:] * xw)
    P = oracle.price(model, S, K, T, r, q, sig, flag)
    for solver in ("lbr", "halley"):
        s, st = fv.implied_vol(model, dev(P), dev(S), dev(K), dev(T), dev(r),
                               flag=dev(flag, torch.int8), q=dev(q) if model == "bsm" else None,
                               solver=solver)
        res = compare_iv(model, solver, P, S, K, T, r, q, flag, host(s), host(st))
        _report("fuzz-far/%s/%s" % (model, solver), res)
        assert len(res["status_bad"]) == 0, res["status_bad"][:5]
        assert len(res["value_bad"]) == 0, (res["value_bad"][:5], res["max_ratio"])
        assert len(res["nan_bad"]) == 0


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_price_fuzz_extreme_ranges(fv, model):
    """fv_price over the fuzz quotes (sigma 1e-4..10, T 1e-6..50, |z| <= 12)
    against the oracle's binary128 price, within 16 u of the price plus its
    first-order sensitivity to rounding every input."""
    _, S, K, T, r, q, sig, flag = _fuzz_quotes(model)
    qd = dev(q) if model == "bsm" else None
    p = host(fv.price(model, dev(S), dev(K), dev(T), dev(r), dev(sig), flag=dev(flag, torch.int8),
                      q=qd))
    po = oracle.price(model, S, K, T, r, q, sig, flag)
    g = oracle.greeks(model, S, K, T, r, q, sig, flag)
    F, D = forward_discount(model, S, T, r, q)
    from scipy.special import ndtr
    with np.errstate(all="ignore"):
        d2 = np.log(F / K) / (sig * np.sqrt(T)) - 0.5 * sig * np.sqrt(T)
        dPdK = -flag * D * ndtr(flag * d2)
        # carry terms: r and q move the forward (and r the discount)
        cond = (np.abs(g["delta"] * S) + np.abs(dPdK * K) + np.abs(g["theta"] * T) +
                np.abs(g["vega"] * sig) + np.abs(g["rho"] * r) + np.abs(T * q * D * F) +
                np.abs(r * T) * np.abs(po) + np.abs(r * T) * D * (F + K))
    tol = 16 * U * (np.abs(po) + cond)
    bad = ~(np.abs(p - po) <= tol)
    print("price-fuzz/%s: max err/tol %.3g" % (model, np.nanmax(np.abs(p - po) / tol)))
    assert bad.sum() == 0, (np.where(bad)[0][:5], p[bad][:5], po[bad][:5])


@pytest.mark.parametrize("solver", ["lbr", "halley"])
def test_subnormal_prices(fv, solver):
    """Out-of-the-money quotes whose price is below the normal binary64 range
    (the accuracy plane's subnormal cells, spread over three models and both
    flags by scaling), and a normalised price that underflows to zero: each
    solved to the oracle's root within the parity tolerance, which is finite
    for every one of them."""
    xs = np.concatenate([[0.0], -np.logspace(-4, np.log10(20.0), 159)])
    ss = np.logspace(-3, np.log10(8.0), 160)
    X, S = (a.ravel() for a in np.meshgrid(xs, ss, indexing="ij"))
    one = np.ones_like(X)
    P = oracle.price("black76", one, np.exp(-X), one, 0 * one, 0.0, S, 1)
    keep = (P > 0) & (P < 2.2250738585072014e-308)
    X, S = X[keep], S[keep]
    m = len(X)
    assert m >= 20
    rng = np.random.default_rng(77)
    for model in ("black76", "bs", "bsm"):
        fl = np.where(rng.random(m) < 0.5, 1, -1).astype(np.int8)
        T = rng.uniform(0.5, 2.0, m)
        r = rng.uniform(0.0, 0.05, m) if model != "black76" else np.zeros(m)
        q = rng.uniform(0.0, 0.03, m) if model == "bsm" else np.zeros(m)
        Sx = np.exp(rng.uniform(np.log(1.0), np.log(1e4), m))
        F, _ = forward_discount(model, Sx, T, r, q)
        # out of the money at |x| for either flag
        K = F * np.exp(-fl * X)
        sig = S / np.sqrt(T)
        Pq = oracle.price(model, Sx, K, T, r, q, sig, fl)
        if model == "black76":
            Sx = np.append(Sx, 1e300)
            K = np.append(K, 1e301)
            T, r, q = np.append(T, 1.0), np.append(r, 0.0), np.append(q, 0.0)
            fl = np.append(fl, np.int8(1))
            Pq = np.append(Pq, 1e-300)
        s, st = fv.implied_vol(model, dev(Pq), dev(Sx), dev(K), dev(T), dev(r),
                               flag=dev(fl, torch.int8), q=dev(q) if model == "bsm" else None,
                               solver=solver)
        res = compare_iv(model, solver, Pq, Sx, K, T, r, q, fl, host(s), host(st))
        _report("subnormal/%s/%s" % (model, solver), res)
        assert res["inf_tol"] == 0
        assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0, (
            res["value_bad"][:5], res["max_ratio"])
        assert res["n_ok"] >= 0.9 * len(Pq)


def test_traces_and_sorted_order(fv):
    """fv_lbr_trace and fv_halley_trace codes are well-formed (LBR: region
    0..3, 2..4 steps; Halley: 1..8 steps, bit 8 for the bisection fallback;
    0xFFFFFFFF exactly where the status is not OK), and solving the quotes
    sorted by either code gives bitwise the same sigma per quote: the sorted
    launches the census counts do the same work as the workload's own order."""
    wl = W.bsm_wide(60_000, seed=17)
    P = assemble_prices(wl)
    ins = [dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r)]
    fl, qq = dev(wl.flag, torch.int8), dev(wl.q)
    for solver, trace in (("lbr", fv.lbr_trace), ("halley", fv.halley_trace)):
        sig, st = fv.implied_vol("bsm", *ins, flag=fl, q=qq, solver=solver)
        code = trace("bsm", *ins, flag=fl, q=qq)
        c = host(code).astype(np.uint32)
        ok = host(st) == 0
        unsolved = c == 0xFFFFFFFF
        # NOT_CONVERGED quotes were solved (their trace is a path code)
        assert np.array_equal(unsolved, np.isin(host(st), [1, 2, 3, 4])), solver
        cs = c[~unsolved]
        if solver == "lbr":
            assert np.all((cs >> 2 & 3) <= 2)
        else:
            assert np.all(((cs & 0xFF) >= 1) & ((cs & 0xFF) <= 8) & ((cs >> 9) == 0))
            assert ((cs >> 8) & 1).mean() < 0.005  # the paper's fallback bound
        order = torch.argsort(code.to(torch.int64))
        sig2, st2 = fv.implied_vol("bsm", *[x.index_select(0, order).contiguous() for x in ins],
                                   flag=fl.index_select(0, order).contiguous(),
                                   q=qq.index_select(0, order).contiguous(), solver=solver)
        inv = torch.empty_like(order)
        inv[order] = torch.arange(order.numel(), device=order.device)
        assert torch.equal(torch.nan_to_num(sig2[inv], -1.0), torch.nan_to_num(sig, -1.0)), solver
        assert torch.equal(st2[inv], st), solver
        assert ok.mean() > 0.97


@pytest.fixture
def halley_limit(fv):
    """Sets the Halley step limit for one test and restores the default."""
    def set_(k):
        fv.set_halley_steps(k)
    yield set_
    fv.set_halley_steps(8)


@pytest.mark.parametrize("limit", [1, 2])
def test_halley_fallback_forced_by_step_limit(fv, halley_limit, limit):
    """The bisection fallback and the Greeks of the quotes it solves, with the
    Halley step limit lowered from the host so that the LDS queue is busy:
    limit 1 sends every solvable quote to it, limit 2 the quotes that need a
    third step (most waves then hold both kinds).  The trace marks exactly
    those quotes; the implied volatility stays within the Halley tolerance of
    the oracle and the fused Greeks within theirs, element by element."""
    wl = W.bsm_diff(50_000, seed=4)
    P = assemble_prices(wl)
    halley_limit(limit)
    assert fv.get_halley_steps() == limit
    q = dev(wl.q)
    code = host(fv.halley_trace("bsm", dev(P), dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r),
                                flag=dev(wl.flag, torch.int8), q=q)).astype(np.uint32)
    solved = code != 0xFFFFFFFF
    fell = ((code[solved] >> 8) & 1) == 1
    steps = code[solved] & 0xFF
    # the first step is at guess precision, so no quote stops before its
    # second: every solvable quote runs the whole (lowered) limit
    assert np.all(steps == limit)
    if limit == 1:
        assert fell.all()
    else:
        assert 0.01 < fell.mean() < 0.99, fell.mean()
    sig, st, gk = run_iv(fv, wl, P, "halley", greeks=True)
    res = compare_iv("bsm", "halley", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag, host(sig),
                     host(st))
    _report("halley-limit-%d" % limit, res)
    assert len(res["status_bad"]) == 0 and len(res["nan_bad"]) == 0
    assert len(res["value_bad"]) == 0, (res["value_bad"][:5], res["max_ratio"])
    st, sg = host(st), host(sig)
    i = np.where(st == 0)[0]
    assert len(i) > 0.999 * len(st)
    bad, worst = greeks_bad("bsm", wl.fs[i], wl.K[i], wl.T[i], wl.r[i], wl.q[i], sg[i],
                            wl.flag[i], {k: host(v)[i] for k, v in gk.items()})
    print("halley-limit-%d greeks: max err/tol %.3g" % (limit, worst))
    for name in GREEK_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])


def test_chains_halley_fallback_matches_flat(fv, halley_limit):
    """Ragged chains through the Halley path with the step limit at 2 (the
    chain kernel's own LDS queue busy): bitwise the flat Halley kernel on
    the expanded arrays under the same limit."""
    ch = W.b76_chains(40, seed=3)
    flat = ch.flatten()
    P = assemble_prices(flat)
    halley_limit(2)
    s_c, st_c = fv.implied_vol_chains(dev(ch.chain_mat_off, torch.int64),
                                      dev(ch.mat_quote_off, torch.int64), dev(ch.F), dev(ch.r),
                                      dev(ch.T), dev(P), dev(ch.K), dev(ch.flag, torch.int8),
                                      solver="halley")
    s_f, st_f = fv.implied_vol("black76", dev(P), dev(flat.fs), dev(flat.K), dev(flat.T),
                               dev(flat.r), flag=dev(flat.flag, torch.int8), solver="halley")
    code = host(fv.halley_trace("black76", dev(P), dev(flat.fs), dev(flat.K), dev(flat.T),
                                dev(flat.r), flag=dev(flat.flag, torch.int8))).astype(np.uint32)
    assert (((code >> 8) & 1) == 1).mean() > 0.01
    assert torch.equal(st_c, st_f)
    assert torch.equal(torch.nan_to_num(s_c, -1.0), torch.nan_to_num(s_f, -1.0))
