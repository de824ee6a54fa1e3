"""Binary32 Halley path (fv_implied_vol_f32) against the oracle.

The oracle solves the same binary32 inputs promoted exactly to binary64.
Contract: |sigma - sigma*| <= max(4e-6 sigma*, 8 u32 sum_X |d sigma/d X| |X|),
u32 = 2^-24.  Statuses agree except within 16 binary32 ulps of the
intrinsic value or the upper bound (decided in binary32 here), and except
quotes outside the solver's domain (normalised price below 2^-100), which
must carry FV_Q_NOT_CONVERGED and NaN."""
import numpy as np
import pytest

import oracle
from _helpers import assemble_prices, boundary_ambiguous, cond_abs, forward_discount
from paper_2604_27210_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_27210_amd as fv
    fv._native.load()
    return fv


def d32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def normalised_beta(model, P, fs, K, T, r, q, flag):
    """beta of the out-of-the-money side in binary64 (domain check only)."""
    F, D = forward_discount(model, fs, T, r, q)
    Pu = P / D
    call = flag > 0
    intrinsic = np.where(call, np.maximum(F - K, 0.0), np.maximum(K - F, 0.0))
    return (Pu - intrinsic) / np.sqrt(F * K)


def check(fv, model, P, fs, K, T, r, q, flag):
    n = P.shape[0]
    f = lambda a: np.ascontiguousarray(np.broadcast_to(a, n), dtype=np.float32)
    A = [f(x) for x in (P, fs, K, T, r, q)]
    sig, st = fv.implied_vol_f32(model, *[d32(a) for a in A[:5]], flag=torch.from_numpy(
        np.ascontiguousarray(flag, dtype=np.int8)).to("cuda"), q=d32(A[5]))
    sig = sig.cpu().numpy().astype(np.float64)
    st = st.cpu().numpy()
    return compare_f32(model, [a.astype(np.float64) for a in A], flag, sig, st)


def compare_f32(model, D, flag, sig, st):
    """The contract above for binary32 inputs D (promoted exactly to float64:
    price, S/F, K, T, r, q), flags, and the GPU's sigma (as float64) and
    status; returns (quotes solved by both, largest error / tolerance)."""
    so, sto = oracle.implied_vol(model, *D, flag)
    dom = (sto == 0) & (st == 5)
    if dom.any():
        beta = normalised_beta(model, *D, flag)[dom]
        assert np.all(beta < 2.0 ** -99), beta.max()
        assert np.all(np.isnan(sig[dom]))
    amb = boundary_ambiguous(model, *D, flag, u=U32)
    bad_status = (sto != st) & ~amb & ~dom
    assert not bad_status.any(), (np.where(bad_status)[0][:5], sto[bad_status][:5], st[bad_status][:5])
    ok = (sto == 0) & (st == 0)
    idx = np.where(ok)[0]
    ca = cond_abs(model, *(x[idx] for x in D), flag[idx])
    tol = np.maximum(4e-6 * so[idx], 8 * U32 * ca)
    err = np.abs(sig[idx] - so[idx])
    ratio = err / tol
    assert np.all(ratio <= 1.0), (ratio.max(), idx[np.argmax(ratio)])
    at = (st == 1) & (sto == 1)
    assert np.all(sig[at] == 0.0)
    assert np.all(np.isnan(sig[(st >= 2) & (st <= 5)]))
    return ok.sum(), ratio.max()


def test_small_batch(fv):
    wl = W.bs_small()
    n, worst = check(fv, "bs", assemble_prices(wl), wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    assert n > 3900 and worst < 0.5


def test_wide_bsm_sample(fv):
    wl = W.bsm_wide(200_000, seed=2)
    n, worst = check(fv, "bsm", assemble_prices(wl), wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    assert n > 150_000 and worst < 0.5


def test_black76_chains_flattened(fv):
    wl = W.b76_chains(60, seed=3).flatten()
    n, worst = check(fv, "black76", assemble_prices(wl), wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    assert n == wl.n and worst < 0.5


def test_domain_edge_and_degenerate(fv):
    # deep out-of-the-money calls spanning beta from 1e-20 to 1e-40 (the
    # domain boundary 2^-100 ~ 7.9e-31 inside), plus degenerate prices
    z = np.linspace(6.0, 14.0, 64)
    T, r, sig = 1.0, 0.0, 0.2
    K = 100.0 * np.exp(z * sig)
    P = oracle.price("black76", np.full(64, 100.0), K, np.full(64, T), np.full(64, r), 0.0,
                     np.full(64, sig), np.ones(64, dtype=np.int8))
    P = np.concatenate([P, [0.0, -1.0, 100.0, np.nan]])
    K = np.concatenate([K, [100.0, 100.0, 100.0, 100.0]])
    n = P.shape[0]
    check(fv, "black76", P, np.full(n, 100.0), K, np.full(n, T), np.full(n, r), np.zeros(n),
          np.ones(n, dtype=np.int8))


def test_empty_and_invalid(fv):
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    sig, st = fv.implied_vol_f32("bs", e, e, e, e, e)
    assert sig.numel() == 0
    with pytest.raises(TypeError):
        fv.implied_vol_f32("bs", torch.ones(4, dtype=torch.float64, device="cuda"), 100.0, 100.0,
                           1.0, 0.0)


@pytest.mark.parametrize("model", ["black76", "bs", "bsm"])
def test_fuzz_extreme_ranges_f32(fv, model):
    """Seeded binary32 quotes beyond the configured workloads: S over six
    decades, T from 1e-6 to 80 years, r up to 0.5, sigma from 1e-3 to 20,
    |z| up to 12 (strikes far enough out that F/K leaves the binary32
    range), against the oracle under the contract above."""
    rng = np.random.default_rng({"black76": 71, "bs": 72, "bsm": 73}[model])
    n = 100_000
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    S = f32(np.exp(rng.uniform(np.log(1e-2), np.log(1e4), n)))
    T = f32(np.exp(rng.uniform(np.log(1e-6), np.log(80.0), n)))
    r = f32(rng.uniform(-0.1, 0.5, n))
    q = f32(rng.uniform(0.0, 0.3, n) if model == "bsm" else np.zeros(n))
    sig = np.exp(rng.uniform(np.log(1e-3), np.log(20.0), n))
    z = rng.uniform(-12, 12, n)
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    with np.errstate(all="ignore"):
        F, D = forward_discount(model, S, T, r, q)
        K = f32(F * np.exp(-z * sig * np.sqrt(T)))
    keep = np.isfinite(K) & (K >= np.finfo(np.float32).tiny) & (K < 1e37)
    S, K, T, r, q, sig, flag = (a[keep] for a in (S, K, T, r, q, sig, flag))
    P = f32(oracle.price(model, S, K, T, r, q, sig, flag))
    keep = np.isfinite(P) & ((P == 0) | (P >= np.finfo(np.float32).tiny))
    S, K, T, r, q, flag, P = (a[keep] for a in (S, K, T, r, q, flag, P))
    n_ok, worst = check(fv, model, P, S, K, T, r, q, flag)
    print("f32 fuzz %s: solved %d of %d, max err/tol %.3g" % (model, n_ok, len(P), worst))
    assert n_ok > 0.5 * len(P)


def test_fallback_forced_by_step_limit_f32(fv):
    """The binary32 bisection fallback, with the Halley step limit lowered to
    1 from the host so that most quotes go through the LDS queue: the
    results still meet the binary32 contract, element by element."""
    wl = W.bsm_wide(100_000, seed=2)
    fv.set_halley_steps(1)
    try:
        n, worst = check(fv, "bsm", assemble_prices(wl), wl.fs, wl.K, wl.T, wl.r, wl.q, wl.flag)
    finally:
        fv.set_halley_steps(8)
    assert n > 75_000 and worst <= 1.0
