"""Differentiable implied volatility on the GPU: the autograd Function's
gradients against the oracle's implicit-function gradient, central finite
differences, and the composite identity d IV(P(sigma))/d sigma = 1."""
import numpy as np
import pytest

import oracle
from paper_2604_27210_amd import workloads as W

from _helpers import (GRAD_NAMES, U, assemble_prices, compare_iv, cond_abs, grad_bad, greek_terms)

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


def test_iv_autograd_matches_oracle_gradient(fv):
    """L = sum(w * sigma) over the differentiation workload (|z| <= 3)."""
    wl = W.bsm_diff(200_000, seed=4)
    P = assemble_prices(wl)
    ins = [dev(P, grad=True), dev(wl.fs, grad=True), dev(wl.K, grad=True), dev(wl.T, grad=True),
           dev(wl.r, grad=True), dev(wl.q, grad=True)]
    sig, st = fv.implied_vol_autograd("bsm", ins[0], ins[1], ins[2], ins[3], ins[4],
                                      flag=dev(wl.flag, torch.int8), q=ins[5])
    w = dev(wl.extra["w"])
    (w * sig).sum().backward()
    st, sg = st.cpu().numpy(), sig.detach().cpu().numpy()
    ok = st == 0
    assert ok.mean() > 0.999
    res = compare_iv("bsm", "lbr", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag, sg, st)
    assert len(res["status_bad"]) == 0 and len(res["value_bad"]) == 0
    got = np.stack([t.grad.cpu().numpy() for t in ins], 1)
    assert np.all(got[~ok] == 0.0)
    i = np.where(ok)[0]
    bad, worst, nonfin = grad_bad("bsm", wl.fs[i], wl.K[i], wl.T[i], wl.r[i], wl.q[i], sg[i],
                                  wl.flag[i], got[i], w=wl.extra["w"][i], P=P[i])
    print("autograd: max err/tol %.3g" % worst)
    assert nonfin == 0
    for name in GRAD_NAMES:
        assert len(bad[name]) == 0, (name, bad[name][:5])


def test_iv_autograd_central_differences(fv):
    """Against FP64 central differences, h = 1e-6 relative (absolute for r
    and q).  A difference quotient carries its own truncation error (the IV
    is strongly curved in the price of deep out-of-the-money quotes), so the
    GPU's quotient is compared with the same quotient of the oracle's exact
    roots, and the GPU's analytic gradient must sit as close to that quotient
    as the oracle's analytic gradient does."""
    wl = W.bsm_diff(20_000, seed=44)
    P = assemble_prices(wl)
    base = dict(price=P, fs=wl.fs, K=wl.K, T=wl.T, r=wl.r, q=wl.q)
    fl = dev(wl.flag, torch.int8)

    def iv(**kw):
        a = dict(base)
        a.update(kw)
        s, st = fv.implied_vol("bsm", dev(a["price"]), dev(a["fs"]), dev(a["K"]), dev(a["T"]),
                               dev(a["r"]), flag=fl, q=dev(a["q"]))
        return s.cpu().numpy()

    def iv_exact(**kw):
        a = dict(base)
        a.update(kw)
        hi, lo, st = oracle.implied_vol("bsm", a["price"], a["fs"], a["K"], a["T"], a["r"], a["q"],
                                        wl.flag, with_residual=True)
        return hi.astype(np.longdouble) + lo

    ins = [dev(base[k], grad=True) for k in ("price", "fs", "K", "T", "r", "q")]
    sig, st = fv.implied_vol_autograd("bsm", *ins[:5], flag=fl, q=ins[5])
    sig.sum().backward()
    ok = st.cpu().numpy() == 0
    go = oracle.iv_grad("bsm", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    # rounding noise of a binary64 IV evaluation (a few ulps of the summed
    # input sensitivities), which a difference quotient divides by 2h
    noise = 8 * U * cond_abs("bsm", P, wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    for j, k in enumerate(("price", "fs", "K", "T", "r", "q")):
        x = base[k]
        h = 1e-6 * (np.abs(x) if k in ("price", "fs", "K", "T") else np.ones_like(x))
        fd = (iv(**{k: x + h}) - iv(**{k: x - h})) / (2 * h)
        fdx = ((iv_exact(**{k: x + h}) - iv_exact(**{k: x - h})) / (2 * h)).astype(float)
        g = ins[j].grad.cpu().numpy()
        # a shifted input can leave the solvable domain (price above its bound)
        m = ok & np.isfinite(fd) & np.isfinite(fdx)
        assert m.mean() > 0.99
        bad = m & ~(np.abs(fd - fdx) <= noise / h + 1e-12 * np.abs(fdx))
        assert bad.sum() == 0, (k, np.where(bad)[0][:5])
        # what the analytic gradient may differ from the quotient by: the
        # quotient's truncation (the oracle's own analytic-vs-quotient gap),
        # plus the gradient's evaluation at the binary64 root instead of the
        # exact one (for ill-conditioned quotes the root's relative error,
        # a few u times the input sensitivities, reaches 1e-9)
        trunc = np.abs(go[:, j] - fdx)
        excess = np.maximum(np.abs(g - fdx) - 1.001 * trunc, 0.0) / np.maximum(np.abs(g), 1e-300)
        assert np.all(excess[m] <= 1e-7), (k, np.where(m & (excess > 1e-7))[0][:5])
        assert np.quantile(excess[m], 0.999) <= 1e-9, k
        rel = np.abs(g - fd) / np.maximum(np.abs(g), 1e-12)
        assert np.median(rel[m]) < 1e-8, k


def test_composite_identity(fv):
    """sigma -> price -> implied vol is the identity; its gradient is 1."""
    wl = W.bsm_diff(100_000, seed=45)
    fl = dev(wl.flag, torch.int8)
    sig = dev(wl.sigma_true, grad=True)
    p = fv.price_autograd("bsm", dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r), sig, flag=fl,
                          q=dev(wl.q))
    iv, st = fv.implied_vol_autograd("bsm", p, dev(wl.fs), dev(wl.K), dev(wl.T), dev(wl.r),
                                     flag=fl, q=dev(wl.q))
    iv.sum().backward()
    ok = st.cpu().numpy() == 0
    g = sig.grad.cpu().numpy()
    # the chain rule gives vega(sigma)/vega(IV): exactly 1 in exact arithmetic,
    # and the ratio of the two vegas at the binary64 root
    ivh = iv.detach().cpu().numpy()
    vs = oracle.greeks("bsm", wl.fs, wl.K, wl.T, wl.r, wl.q, wl.sigma_true, wl.flag)["vega"]
    vi = oracle.greeks("bsm", wl.fs, wl.K, wl.T, wl.r, wl.q, ivh, wl.flag)["vega"]
    bad = ok & ~(np.abs(g - vs / vi) <= 1e-10 * (vs / vi))
    assert bad.sum() == 0, (bad.sum(), np.where(bad)[0][:5], g[bad][:5], wl.sigma_true[bad][:5])
    assert np.median(np.abs(g[ok] - 1.0)) < 1e-12
    np.testing.assert_allclose(iv.detach().cpu().numpy()[ok], wl.sigma_true[ok], rtol=1e-6)


def test_price_adjoint_matches_oracle_greeks(fv):
    wl = W.bsm_diff(50_000, seed=46)
    fl = dev(wl.flag, torch.int8)
    ins = [dev(a, grad=True) for a in (wl.fs, wl.K, wl.T, wl.r, wl.q, wl.sigma_true)]
    p = fv.price_autograd("bsm", ins[0], ins[1], ins[2], ins[3], ins[5], flag=fl, q=ins[4])
    p.sum().backward()
    S, K, T, r, q, sg, fl_h = wl.fs, wl.K, wl.T, wl.r, wl.q, wl.sigma_true, wl.flag
    g = oracle.greeks("bsm", S, K, T, r, q, sg, fl_h)
    # dP/dK and dP/dq at fixed sigma from the oracle's gradient formula:
    # -vega d sigma/dX
    ga = oracle.iv_grad_at("bsm", S, K, T, r, q, sg, fl_h)
    P = oracle.price("bsm", S, K, T, r, q, sg, fl_h)
    kappa, theta_terms = greek_terms("bsm", S, K, T, r, q, sg, fl_h, P)
    refs = ((ins[0], g["delta"], np.abs(g["delta"])), (ins[1], -ga[:, 2] * g["vega"], np.abs(ga[:, 2] * g["vega"])),
            (ins[2], -g["theta"], theta_terms), (ins[3], g["rho"], np.abs(g["rho"])),
            (ins[4], -ga[:, 5] * g["vega"], np.abs(ga[:, 5] * g["vega"])),
            (ins[5], g["vega"], np.abs(g["vega"])))
    for t, ref, scale in refs:
        a = t.grad.cpu().numpy()
        tol = 64 * U * kappa * scale + 1e-300
        bad = ~(np.abs(a - ref) <= tol)
        assert bad.sum() == 0, (np.where(bad)[0][:5], a[bad][:5], ref[bad][:5])


def test_autograd_with_fused_greeks(fv):
    """greeks=True returns the fused launch's Greeks (bitwise those of the
    plain call) and leaves sigma and every gradient unchanged."""
    wl = W.bsm_diff(30_000, seed=47)
    P = assemble_prices(wl)
    fl = dev(wl.flag, torch.int8)
    grads = []
    for greeks in (False, True):
        ins = [dev(a, grad=True) for a in (P, wl.fs, wl.K, wl.T, wl.r, wl.q)]
        out = fv.implied_vol_autograd("bsm", *ins[:5], flag=fl, q=ins[5], greeks=greeks)
        (dev(wl.extra["w"]) * out[0]).sum().backward()
        grads.append([t.grad.clone() for t in ins] + [out[0].detach()])
        if greeks:
            gk = out[2]
            assert set(gk) == {"delta", "gamma", "vega", "theta", "rho"}
            assert not any(t.requires_grad for t in gk.values())
            _, _, ref = fv.implied_vol("bsm", *[t.detach() for t in ins[:5]], flag=fl,
                                       q=ins[5].detach(), greeks=True)
            for k in gk:
                assert torch.equal(torch.nan_to_num(gk[k], nan=-1.0), torch.nan_to_num(ref[k], nan=-1.0)), k
    for a, b in zip(*grads):
        assert torch.equal(torch.nan_to_num(a, nan=-1.0), torch.nan_to_num(b, nan=-1.0))


def test_scalar_inputs_get_summed_gradients(fv):
    """A 0-dim tensor broadcast to every quote (a shared r and T here) gets
    the sum over the quotes of the per-quote gradient, in the IV and in the
    price adjoint; the per-quote run on the same values gives the rows."""
    wl = W.bsm_diff(20_000, seed=48)
    n = wl.n
    T0, r0 = 0.75, 0.02
    fl = dev(wl.flag, torch.int8)
    P = oracle.price("bsm", wl.fs, wl.K, T0, r0, wl.q, wl.sigma_true, wl.flag)
    # per-quote tensors holding the shared values
    ins = [dev(P, grad=True), dev(wl.fs, grad=True), dev(wl.K, grad=True),
           dev(np.full(n, T0), grad=True), dev(np.full(n, r0), grad=True), dev(wl.q, grad=True)]
    sig, st = fv.implied_vol_autograd("bsm", *ins[:5], flag=fl, q=ins[5])
    w = dev(wl.extra["w"])
    (w * sig).sum().backward()
    # 0-dim tensors for T and r, on the GPU and on the CPU
    for where in ("cuda", "cpu"):
        Ts = torch.tensor(T0, dtype=torch.float64, device=where, requires_grad=True)
        rs = torch.tensor(r0, dtype=torch.float64, device=where, requires_grad=True)
        ins2 = [dev(P, grad=True), dev(wl.fs), dev(wl.K), Ts, rs, dev(wl.q)]
        sig2, st2 = fv.implied_vol_autograd("bsm", *ins2[:5], flag=fl, q=ins2[5])
        # the same solve (unsolved quotes are NaN in both, which torch.equal
        # would count as a difference)
        assert torch.equal(st2, st)
        assert torch.equal(torch.isnan(sig2), torch.isnan(sig))
        ok = ~torch.isnan(sig)
        assert torch.allclose(sig2.detach()[ok], sig.detach()[ok], rtol=1e-15, atol=0.0)
        (w * sig2).sum().backward()
        assert Ts.grad is not None and rs.grad is not None
        assert Ts.grad.device.type == where and Ts.grad.dim() == 0
        for t0, t in ((ins[3], Ts), (ins[4], rs)):
            ref = t0.grad.sum().item()
            assert abs(t.grad.item() - ref) <= 1e-12 * t0.grad.abs().sum().item(), (where, t.grad, ref)
        assert torch.allclose(ins2[0].grad, ins[0].grad, rtol=1e-13, atol=0.0)
    # the price adjoint: a shared sigma and r
    sg = torch.tensor(0.3, dtype=torch.float64, device="cuda", requires_grad=True)
    rs = torch.tensor(r0, dtype=torch.float64, device="cuda", requires_grad=True)
    p = fv.price_autograd("bsm", dev(wl.fs), dev(wl.K), dev(np.full(n, T0)), rs, sg, flag=fl,
                          q=dev(wl.q))
    p.sum().backward()
    g = oracle.greeks("bsm", wl.fs, wl.K, T0, r0, wl.q, 0.3, wl.flag)
    for t, name in ((sg, "vega"), (rs, "rho")):
        assert abs(t.grad.item() - g[name].sum()) <= 1e-10 * np.abs(g[name]).sum(), name
