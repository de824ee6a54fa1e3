"""Pins of the binary128 oracle against facts other than its own formulas.

Every check here comes from something independent of ``oracle/fv_oracle.c``:
a textbook worked example, the risk-neutral expectation evaluated by
numerical quadrature (mpmath), closed forms through library routines
(scipy ``erf``/``erfinv``), no-arbitrage identities, limits, brute-force
bisection, central finite differences and scaling invariants.  Each is chosen
so that a plausible slip in the oracle -- a dropped term, a wrong sign or
index, a swapped operand, a put branch with the call's sign -- fails at least
one of them.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
from scipy import special

HERE = os.path.dirname(os.path.abspath(__file__))
MODELS = ["black76", "bs", "bsm"]


def _rand_quotes(rng, n, model, zmax=3.0):
    S = rng.uniform(20, 200, n)
    T = np.exp(rng.uniform(np.log(0.02), np.log(3.0), n))
    r = rng.uniform(-0.01, 0.08, n)
    q = rng.uniform(0.0, 0.05, n) if model == "bsm" else np.zeros(n)
    sig = np.exp(rng.uniform(np.log(0.05), np.log(1.5), n))
    z = rng.uniform(-zmax, zmax, n)
    carry = (r - q) if model == "bsm" else (r if model == "bs" else 0.0)
    F = S * np.exp(carry * T)
    K = F * np.exp(-z * sig * np.sqrt(T))
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    return S, K, T, r, q, sig, flag


def _forward_discount(model, fs, T, r, q):
    if model == "black76":
        return mp.mpf(fs), mp.exp(-mp.mpf(r) * T)
    carry = (mp.mpf(r) - mp.mpf(q)) if model == "bsm" else mp.mpf(r)
    return mp.mpf(fs) * mp.exp(carry * mp.mpf(T)), mp.exp(-mp.mpf(r) * mp.mpf(T))


def _price_by_quadrature(model, fs, K, T, r, q, sig, theta):
    """D * E[(theta (F_T - K))^+], F_T = F exp(s W - s^2/2), W ~ N(0,1),
    integrated numerically -- the risk-neutral definition of the price."""
    F, D = _forward_discount(model, fs, T, r, q)
    K = mp.mpf(K)
    s = mp.mpf(sig) * mp.sqrt(mp.mpf(T))
    wstar = (mp.log(K / F) + s * s / 2) / s
    dens = lambda w: mp.exp(-w * w / 2) / mp.sqrt(2 * mp.pi)
    if theta > 0:
        f = lambda w: (F * mp.exp(s * w - s * s / 2) - K) * dens(w)
        val = mp.quad(f, [wstar, wstar + 1, wstar + 8, mp.inf])
    else:
        f = lambda w: (K - F * mp.exp(s * w - s * s / 2)) * dens(w)
        val = mp.quad(f, [-mp.inf, wstar - 8, wstar - 1, wstar])
    return D * val


def test_textbook_worked_example(orc):
    g = json.load(open(os.path.join(HERE, "golden", "hull_bsm_example.json")))
    a = g["inputs"]
    c, p = orc.price("bsm", a["S"], a["K"], a["T"], a["r"], 0.0, a["sigma"], [1, -1])
    assert round(c, 2) == g["printed"]["call"]
    assert round(p, 2) == g["printed"]["put"]
    # the same example through plain Black-Scholes (q = 0) and Black-76 on F
    c2 = orc.price("bs", a["S"], a["K"], a["T"], a["r"], 0.0, a["sigma"], 1)[0]
    F = a["S"] * math.exp(a["r"] * a["T"])
    c3 = orc.price("black76", F, a["K"], a["T"], a["r"], 0.0, a["sigma"], 1)[0]
    assert abs(c2 - c) <= 1e-14 * c and abs(c3 - c) <= 1e-13 * c


@pytest.mark.parametrize("model", MODELS)
def test_price_equals_risk_neutral_quadrature(orc, model):
    mp.mp.dps = 30
    rng = np.random.default_rng(11 + MODELS.index(model))
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 24, model, zmax=4.0)
    got = orc.price(model, S, K, T, r, q, sig, flag)
    for i in range(len(S)):
        ref = _price_by_quadrature(model, S[i], K[i], T[i], r[i], q[i], sig[i], flag[i])
        assert abs(got[i] - float(ref)) <= 4e-15 * float(ref), (i, got[i], ref)


@pytest.mark.parametrize("model", MODELS)
def test_put_call_parity_and_limits(orc, model):
    mp.mp.dps = 40  # the parity residual is compared at 1e-28 relative
    rng = np.random.default_rng(21)
    S, K, T, r, q, sig, _ = _rand_quotes(rng, 500, model)
    ch, cl = orc.price(model, S, K, T, r, q, sig, 1, with_residual=True)
    ph, pl = orc.price(model, S, K, T, r, q, sig, -1, with_residual=True)
    for i in range(0, 500, 25):
        F, D = _forward_discount(model, S[i], T[i], r[i], q[i])
        lhs = (mp.mpf(ch[i]) + cl[i]) - (mp.mpf(ph[i]) + pl[i])
        rhs = D * (F - mp.mpf(K[i]))
        assert abs(lhs - rhs) <= 1e-28 * (abs(ch[i]) + abs(ph[i]))
    # sigma -> 0: discounted intrinsic; sigma -> infinity: discounted maximum
    lo_c = orc.price(model, S, K, T, r, q, 1e-9, 1)
    lo_p = orc.price(model, S, K, T, r, q, 1e-9, -1)
    hi_c = orc.price(model, S, K, T, r, q, 1e3, 1)
    hi_p = orc.price(model, S, K, T, r, q, 1e3, -1)
    carry = (r - q) if model == "bsm" else (r if model == "bs" else 0.0)
    F = S * np.exp(carry * T)
    D = np.exp(-r * T)
    np.testing.assert_allclose(lo_c, D * np.maximum(F - K, 0), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(lo_p, D * np.maximum(K - F, 0), rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(hi_c, D * F, rtol=1e-12)
    np.testing.assert_allclose(hi_p, D * K, rtol=1e-12)


@pytest.mark.parametrize("model", MODELS)
def test_atm_closed_form_erf(orc, model):
    # F = K: undiscounted call = put = F erf(s / (2 sqrt 2))
    rng = np.random.default_rng(31)
    T = rng.uniform(0.01, 4, 200)
    r = rng.uniform(0, 0.05, 200)
    q = rng.uniform(0, 0.04, 200) if model == "bsm" else np.zeros(200)
    sig = rng.uniform(0.01, 2.0, 200)
    S = np.full(200, 100.0)
    carry = (r - q) if model == "bsm" else (r if model == "bs" else 0.0)
    F = S * np.exp(carry * T)
    D = np.exp(-r * T)
    for fl in (1, -1):
        got = orc.price(model, S, F, T, r, q, sig, fl)
        ref = D * F * special.erf(sig * np.sqrt(T) / (2 * np.sqrt(2)))
        np.testing.assert_allclose(got, ref, rtol=2e-14)


def test_dividend_and_model_equivalences(orc):
    rng = np.random.default_rng(41)
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 300, "bsm")
    bsm = orc.price("bsm", S, K, T, r, q, sig, flag)
    bs_on_prepaid = orc.price("bs", S * np.exp(-q * T), K, T, r, 0.0, sig, flag)
    np.testing.assert_allclose(bsm, bs_on_prepaid, rtol=1e-12)
    b76 = orc.price("black76", S * np.exp((r - q) * T), K, T, r, 0.0, sig, flag)
    np.testing.assert_allclose(bsm, b76, rtol=1e-12)
    # Black-76 ignores q; plain Black-Scholes ignores q
    np.testing.assert_array_equal(orc.price("black76", S, K, T, r, q, sig, flag),
                                  orc.price("black76", S, K, T, r, 0.0 * q, sig, flag))
    np.testing.assert_array_equal(orc.price("bs", S, K, T, r, q, sig, flag),
                                  orc.price("bs", S, K, T, r, 0.0 * q, sig, flag))


# ---------------------------------------------------------------- normalised b
def test_normalised_black_is_integral_of_its_derivative(orc):
    """For x <= 0 the call b(x, s) = int_0^s b'(u) du with the positive
    integrand b'(u) = exp(-(x^2/u^2 + u^2/4)/2)/sqrt(2 pi): no cancellation,
    no error function.  Integrated over v = 1/u, where it is a Gaussian tail."""
    mp.mp.dps = 40
    rng = np.random.default_rng(51)
    xs = -np.exp(rng.uniform(np.log(1e-3), np.log(30.0), 30))
    hs = -np.exp(rng.uniform(np.log(0.05), np.log(8.0), 30))
    ss = xs / hs
    got = orc.normalised_black(xs, ss, 1)
    for x, s, g in zip(xs, ss, got):
        X = mp.mpf(x)
        f = lambda v: mp.exp(-X * X * v * v / 2 - 1 / (8 * v * v)) / (mp.sqrt(2 * mp.pi) * v * v)
        a = 1 / mp.mpf(s)
        d = 1 / (X * X * a + 1)  # decay length of the integrand near v = a
        ref = mp.quad(f, [a + k * d for k in range(60)] + [mp.inf])
        assert abs(g - float(ref)) <= 4e-15 * float(ref), (x, s, g, ref)


def _mills_ratio_cf(z, terms=400):
    """Laplace's continued fraction for the Mills ratio (1 - Phi(z))/phi(z),
    z > 0: 1/(z + 1/(z + 2/(z + 3/(z + ...)))), evaluated bottom-up."""
    acc = mp.mpf(0)
    for k in range(terms, 0, -1):
        acc = k / (z + acc)
    return 1 / (z + acc)


def test_normalised_black_deep_wing_continued_fraction(orc):
    """Deep out-of-the-money: b = b'(s) [R(-(h+t)) - R(t-h)] with R the Mills
    ratio from Laplace's continued fraction (independent of erfc)."""
    mp.mp.dps = 60
    rng = np.random.default_rng(53)
    hs = -rng.uniform(8.0, 36.0, 40)
    ts = np.exp(rng.uniform(np.log(1e-4), np.log(3.0), 40))
    xs = 2 * hs * ts
    ss = 2 * ts
    got = orc.normalised_black(xs, ss, 1)
    for x, s, g in zip(xs, ss, got):
        h, t = mp.mpf(x) / mp.mpf(s), mp.mpf(s) / 2
        bp = mp.exp(-(h * h + t * t) / 2) / mp.sqrt(2 * mp.pi)
        ref = bp * (_mills_ratio_cf(-(h + t)) - _mills_ratio_cf(t - h))
        assert abs(g - float(ref)) <= 4e-15 * float(ref), (x, s, g, ref)


def test_normalised_black_identities(orc):
    rng = np.random.default_rng(52)
    x = rng.uniform(-5, 5, 400)
    s = np.exp(rng.uniform(np.log(1e-3), np.log(8), 400))
    c = orc.normalised_black(x, s, 1)
    p = orc.normalised_black(x, s, -1)
    # call-put parity and the reflection symmetry b(x,s,theta) = b(-x,s,-theta)
    np.testing.assert_allclose(c - p, np.exp(x / 2) - np.exp(-x / 2), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(orc.normalised_black(-x, s, -1), c, rtol=1e-15)
    # at the money: b(0, s) = erf(s / (2 sqrt 2))
    np.testing.assert_allclose(orc.normalised_black(0.0, s, 1),
                               special.erf(s / (2 * np.sqrt(2))), rtol=1e-15)
    # price = D sqrt(F K) b(ln(F/K), sigma sqrt(T))
    F = 100 * np.exp(x / 3)
    K = 100.0
    T = 0.7
    sig = s / np.sqrt(T)
    pr = orc.price("black76", F, K, T, 0.03, 0.0, sig, 1)
    xr = np.log(F / K)  # rounded here; keep rows whose price is insensitive to that
    m = np.abs(xr / s) < 5
    np.testing.assert_allclose(pr[m], (np.exp(-0.03 * T) * np.sqrt(F * K) *
                               orc.normalised_black(xr, s, 1))[m], rtol=1e-13)


# ---------------------------------------------------------------- implied vol
@pytest.mark.parametrize("model", MODELS)
def test_iv_round_trip_and_parity(orc, model):
    rng = np.random.default_rng(61 + MODELS.index(model))
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 2000, model, zmax=5.0)
    P = orc.price(model, S, K, T, r, q, sig, flag)
    iv, st = orc.implied_vol(model, P, S, K, T, r, q, flag)
    ok = st == 0
    assert ok.mean() > 0.99
    # backward error: re-pricing the root gives back the input price
    P2 = orc.price(model, S[ok], K[ok], T[ok], r[ok], q[ok], iv[ok], flag[ok])
    assert np.all(np.abs(P2 - P[ok]) <= 4 * np.spacing(P[ok]))
    # forward error, on well-conditioned quotes, against the sigma priced
    g = orc.greeks(model, S, K, T, r, q, sig, flag)
    kappa = P / (sig * g["vega"])
    good = ok & (kappa * 2.0 ** -53 < 1e-14)
    np.testing.assert_allclose(iv[good], sig[good], rtol=2e-13)
    # call and put prices of the same sigma invert to the same sigma
    Pc = orc.price(model, S, K, T, r, q, sig, 1)
    Pp = orc.price(model, S, K, T, r, q, sig, -1)
    ivc, stc = orc.implied_vol(model, Pc, S, K, T, r, q, 1)
    ivp, stp = orc.implied_vol(model, Pp, S, K, T, r, q, -1)
    gc = orc.greeks(model, S, K, T, r, q, sig, 1)
    kc = np.maximum(Pc, Pp) / (sig * gc["vega"])  # the in-the-money side is the worse
    both = (stc == 0) & (stp == 0) & (kc * 2.0 ** -53 < 1e-14)
    np.testing.assert_allclose(ivc[both], ivp[both], rtol=2e-13)


def test_iv_round_trip_deep_wings(orc):
    """Deep out-of-the-money quotes (h = ln(F/K)/s down to -36, prices far
    below 1e-100): the root still re-prices to the input price, and the
    iteration never hits its cap."""
    rng = np.random.default_rng(65)
    n = 3000
    h = -np.exp(rng.uniform(np.log(1e-3), np.log(36), n))
    t = np.exp(rng.uniform(np.log(1e-4), np.log(4), n))
    F = 100.0
    K = F * np.exp(-2 * h * t)
    T = rng.uniform(0.01, 3, n)
    sig = 2 * t / np.sqrt(T)
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    P = orc.price("black76", F, K, T, 0.0, 0.0, sig, flag)
    iv, st = orc.implied_vol("black76", P, F, K, T, 0.0, 0.0, flag)
    assert not np.any(st == orc.ST_ROOT_CAP)
    ok = st == 0
    assert ok.mean() > 0.9
    P2 = orc.price("black76", F, K[ok], T[ok], 0.0, 0.0, iv[ok], flag[ok])
    # re-pricing error is the price's own sensitivity to one ulp of sigma
    vega = orc.greeks("black76", F, K[ok], T[ok], 0.0, 0.0, iv[ok], flag[ok])["vega"]
    assert np.all(np.abs(P2 - P[ok]) <= 4 * np.spacing(P[ok]) + 2 * vega * np.spacing(iv[ok]))


def test_iv_atm_closed_form_erfinv(orc):
    # Black-76, F = K: P = D F erf(s / (2 sqrt 2))  =>  s = 2 sqrt(2) erfinv(P/(D F))
    rng = np.random.default_rng(71)
    n = 300
    F = rng.uniform(10, 500, n)
    T = rng.uniform(0.05, 3, n)
    r = rng.uniform(0, 0.05, n)
    beta = rng.uniform(1e-4, 0.99, n)
    P = np.exp(-r * T) * F * beta
    iv, st = orc.implied_vol("black76", P, F, F, T, r, 0.0, 1)
    assert np.all(st == 0)
    Pu = P / np.exp(-r * T)
    ref = 2 * np.sqrt(2) * special.erfinv(Pu / F) / np.sqrt(T)
    np.testing.assert_allclose(iv, ref, rtol=1e-13)


def test_iv_brute_force_bisection(orc):
    """Bisection on the quadrature price (no closed form, no Newton)."""
    mp.mp.dps = 25
    rng = np.random.default_rng(81)
    for model in MODELS:
        S, K, T, r, q, sig, flag = _rand_quotes(rng, 2, model, zmax=3.0)
        P = orc.price(model, S, K, T, r, q, sig, flag)
        iv, st = orc.implied_vol(model, P, S, K, T, r, q, flag)
        for i in range(2):
            lo, hi = mp.mpf("1e-4"), mp.mpf(5)
            for _ in range(48):
                mid = (lo + hi) / 2
                v = _price_by_quadrature(model, S[i], K[i], T[i], r[i], q[i], mid, flag[i])
                if v < P[i]:
                    lo = mid
                else:
                    hi = mid
            assert abs(iv[i] - float((lo + hi) / 2)) <= 1e-12 * iv[i]


def test_iv_status_codes_and_limits(orc):
    S, K, T, r, q = 100.0, 90.0, 0.5, 0.03, 0.01
    F = S * math.exp((r - q) * T)
    D = math.exp(-r * T)
    intrinsic_c = D * (F - K)
    P = np.array([intrinsic_c * 0.999, D * F * 1.0000001, 5.0, np.nan, 12.0, 12.0])
    Ks = np.array([K, K, K, K, -1.0, K])
    Ts = np.array([T, T, T, T, T, 0.0])
    iv, st = orc.implied_vol("bsm", P, S, Ks, Ts, r, q, 1)
    assert list(st) == [2, 3, 2, 4, 4, 4]
    assert np.all(np.isnan(iv))
    # an out-of-the-money put exactly at zero price is at intrinsic: sigma = 0
    iv0, st0 = orc.implied_vol("bsm", 0.0, S, K, T, r, q, -1)
    assert st0[0] == 1 and iv0[0] == 0.0
    # monotone in the price, tends to 0 at intrinsic and grows without bound at the maximum
    Ps = np.linspace(intrinsic_c * (1 + 1e-9), D * F * (1 - 1e-9), 400)
    iv, st = orc.implied_vol("bsm", Ps, S, K, T, r, q, 1)
    assert np.all(st == 0) and np.all(np.diff(iv) > 0)
    assert iv[0] < 0.05 and iv[-1] > 10


# ---------------------------------------------------------------- Greeks
def _fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


@pytest.mark.parametrize("model", MODELS)
def test_greeks_match_finite_differences(orc, model):
    rng = np.random.default_rng(91 + MODELS.index(model))
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 200, model, zmax=2.5)

    def P(**kw):
        a = dict(fs=S, K=K, T=T, r=r, q=q, sigma=sig)
        a.update(kw)
        hi, lo = orc.price(model, a["fs"], a["K"], a["T"], a["r"], a["q"], a["sigma"], flag,
                           with_residual=True)
        return hi.astype(np.longdouble) + lo

    g = orc.greeks(model, S, K, T, r, q, sig, flag)
    hS = 1e-7 * S
    d = (P(fs=S + hS) - P(fs=S - hS)) / (2 * hS)
    np.testing.assert_allclose(g["delta"], d.astype(float), rtol=1e-7, atol=1e-12)
    # gamma as the central difference of the oracle's own delta
    hG = 1e-5 * S
    dp = orc.greeks(model, S + hG, K, T, r, q, sig, flag)["delta"]
    dm = orc.greeks(model, S - hG, K, T, r, q, sig, flag)["delta"]
    np.testing.assert_allclose(g["gamma"], (dp - dm) / (2 * hG), rtol=1e-5, atol=1e-10)
    hs = 1e-6 * sig
    v = (P(sigma=sig + hs) - P(sigma=sig - hs)) / (2 * hs)
    np.testing.assert_allclose(g["vega"], v.astype(float), rtol=1e-7, atol=1e-12)
    hT = 1e-6 * T
    th = -(P(T=T + hT) - P(T=T - hT)) / (2 * hT)
    np.testing.assert_allclose(g["theta"], th.astype(float), rtol=1e-6, atol=1e-9)
    hr = 1e-6
    rh = (P(r=r + hr) - P(r=r - hr)) / (2 * hr)
    np.testing.assert_allclose(g["rho"], rh.astype(float), rtol=1e-6, atol=1e-9)


def test_greeks_identities(orc):
    rng = np.random.default_rng(101)
    S, K, T, r, q, sig, _ = _rand_quotes(rng, 500, "bsm")
    gc = orc.greeks("bsm", S, K, T, r, q, sig, 1)
    gp = orc.greeks("bsm", S, K, T, r, q, sig, -1)
    np.testing.assert_allclose(gc["delta"] - gp["delta"], np.exp(-q * T), rtol=1e-13)
    np.testing.assert_allclose(gc["gamma"], gp["gamma"], rtol=1e-13)
    np.testing.assert_allclose(gc["vega"], gp["vega"], rtol=1e-13)
    # Black-Scholes-Merton PDE: theta = r P - (r - q) S delta - sigma^2 S^2 gamma / 2
    for fl, g in ((1, gc), (-1, gp)):
        P = orc.price("bsm", S, K, T, r, q, sig, fl)
        pde = r * P - (r - q) * S * g["delta"] - 0.5 * sig ** 2 * S ** 2 * g["gamma"]
        assert np.all(np.abs(g["theta"] - pde) <= 1e-10 * (np.abs(r * P) + np.abs(S * g["delta"])
                                                           + sig ** 2 * S ** 2 * g["gamma"]))
    # Black-76: delta_c - delta_p = D; rho = -T P
    F = S
    bc = orc.greeks("black76", F, K, T, r, 0.0, sig, 1)
    bp = orc.greeks("black76", F, K, T, r, 0.0, sig, -1)
    np.testing.assert_allclose(bc["delta"] - bp["delta"], np.exp(-r * T), rtol=1e-13)
    np.testing.assert_allclose(bc["rho"], -T * orc.price("black76", F, K, T, r, 0, sig, 1),
                               rtol=1e-14)


# ---------------------------------------------------------------- IV gradient
@pytest.mark.parametrize("model", MODELS)
def test_iv_gradient_matches_finite_differences(orc, model):
    rng = np.random.default_rng(111 + MODELS.index(model))
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 150, model, zmax=2.5)
    P = orc.price(model, S, K, T, r, q, sig, flag)
    grad = orc.iv_grad(model, P, S, K, T, r, q, flag)

    def IV(**kw):
        a = dict(price=P, fs=S, K=K, T=T, r=r, q=q)
        a.update(kw)
        hi, lo, st = orc.implied_vol(model, a["price"], a["fs"], a["K"], a["T"], a["r"], a["q"],
                                     flag, with_residual=True)
        assert np.all(st == 0)
        return hi.astype(np.longdouble) + lo

    steps = [("price", P, 1e-7 * P), ("fs", S, 1e-7 * S), ("K", K, 1e-7 * K),
             ("T", T, 1e-7 * T), ("r", r, 1e-7 * np.ones_like(r))]
    if model == "bsm":
        steps.append(("q", q, 1e-7 * np.ones_like(q)))
    for j, (name, x, h) in enumerate(steps):
        fd = ((IV(**{name: x + h}) - IV(**{name: x - h})) / (2 * h)).astype(float)
        np.testing.assert_allclose(grad[:, j], fd, rtol=1e-6, atol=1e-9, err_msg=name)
    if model != "bsm":
        assert np.all(grad[:, 5] == 0)


def test_iv_gradient_invariants(orc):
    rng = np.random.default_rng(121)
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 400, "bsm", zmax=3.0)
    P = orc.price("bsm", S, K, T, r, q, sig, flag)
    g = orc.iv_grad("bsm", P, S, K, T, r, q, flag)
    vega = orc.greeks("bsm", S, K, T, r, q, sig, flag)["vega"]
    # d sigma / d P * vega = 1 (the composite IV(P(sigma)) has unit slope)
    np.testing.assert_allclose(g[:, 0] * vega, 1.0, rtol=1e-10)
    # homogeneity: sigma is unchanged by scaling price, spot and strike together
    euler = g[:, 0] * P + g[:, 1] * S + g[:, 2] * K
    scale = np.abs(g[:, 0] * P) + np.abs(g[:, 1] * S) + np.abs(g[:, 2] * K)
    assert np.all(np.abs(euler) <= 1e-10 * scale)


# ------------------------------------------- relative sensitivities of the IV
@pytest.mark.parametrize("model", MODELS)
def test_iv_rel_sens_matches_log_differences(orc, model):
    """X d sigma/d X against central differences of the exact root in ln X
    (r and q: r d sigma/d r from absolute steps), normal-range prices."""
    rng = np.random.default_rng(131 + MODELS.index(model))
    S, K, T, r, q, sig, flag = _rand_quotes(rng, 120, model, zmax=2.5)
    P = orc.price(model, S, K, T, r, q, sig, flag)
    e = orc.iv_rel_sens(model, P, S, K, T, r, q, flag)

    def IV(**kw):
        a = dict(price=P, fs=S, K=K, T=T, r=r, q=q)
        a.update(kw)
        hi, lo, st = orc.implied_vol(model, a["price"], a["fs"], a["K"], a["T"], a["r"], a["q"],
                                     flag, with_residual=True)
        assert np.all(st == 0)
        return hi.astype(np.longdouble) + lo

    # steps in ln X as actually taken (the bumped inputs are rounded)
    h = 1e-7
    L = np.longdouble
    for j, name in enumerate(("price", "fs", "K", "T")):
        x = dict(price=P, fs=S, K=K, T=T)[name]
        xp, xm = x * np.exp(h), x * np.exp(-h)
        dl = np.log(xp.astype(L)) - np.log(xm.astype(L))
        fd = ((IV(**{name: xp}) - IV(**{name: xm})) / dl).astype(float)
        np.testing.assert_allclose(e[:, j], fd, rtol=1e-5, atol=1e-10, err_msg=name)
    for j, name in ((4, "r"), (5, "q")):
        x = dict(r=r, q=q)[name]
        fd = (x * (IV(**{name: x + h}) - IV(**{name: x - h})) / (2 * h)).astype(float)
        np.testing.assert_allclose(e[:, j], fd, rtol=1e-5, atol=1e-10, err_msg=name)
    if model != "bsm":
        assert np.all(e[:, 5] == 0)


def _subnormal_price_cells(orc, r=0.0):
    """Black-76 calls with F = 1, K = e^{-x}, T = 1 whose price lies below the
    smallest normal binary64 number (deep out of the money): vega there is
    below the binary64 range as well, and 1/vega overflows."""
    xs = -np.linspace(5.0, 20.0, 61)
    ss = np.exp(np.linspace(np.log(0.05), np.log(1.5), 61))
    X, Sg = (a.ravel() for a in np.meshgrid(xs, ss, indexing="ij"))
    K = np.exp(-X)
    one = np.ones_like(X)
    P = orc.price("black76", one, K, one, r * one, 0.0, Sg, 1)
    keep = (P > 0) & (P < 2.2250738585072014e-308)
    return X[keep], K[keep], P[keep]


@pytest.mark.parametrize("r", [0.0, 0.03])
def test_iv_rel_sens_subnormal_prices(orc, r):
    """Where the price is subnormal, the sensitivities stay finite and obey
    what the mathematics fixes:
      * Euler: the IV is homogeneous of degree 0 in (price, F, K), so the
        three signed relative sensitivities sum to zero;
      * Black-76: sigma sqrt(T) depends on T only through the undiscounted
        price P e^{rT}, so T dsigma/dT = -sigma/2 + r T e_P and
        r dsigma/dr = r T e_P;
      * e_P = P dsigma/dP = (b/b')/sqrt(T) at the root, with
        b/b' = sqrt(pi/2) [erfcx(-(h+t)/sqrt2) - erfcx((t-h)/sqrt2)]
        evaluated in mpmath at 60 digits."""
    x, K, P = _subnormal_price_cells(orc, r)
    assert len(x) >= 20
    one = np.ones_like(x)
    e = orc.iv_rel_sens("black76", P, one, K, one, r * one, 0.0, 1)
    so, st = orc.implied_vol("black76", P, one, K, one, r * one, 0.0, 1)
    assert np.all(st == 0) and np.all(np.isfinite(e[:, :5]))
    # the binary64 gradient overflows here: the reason for this entry point
    g = orc.iv_grad("black76", P, one, K, one, r * one, 0.0, 1)
    assert np.all(~np.isfinite(g[:, 0]) | (np.abs(g[:, 0]) > 1e300))
    scale = np.abs(e[:, 0]) + np.abs(e[:, 1]) + np.abs(e[:, 2])
    assert np.all(np.abs(e[:, 0] + e[:, 1] + e[:, 2]) <= 1e-13 * scale)
    np.testing.assert_allclose(e[:, 3], -so / 2 + r * e[:, 0], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(e[:, 4], r * e[:, 0], rtol=1e-12, atol=0)
    mp.mp.dps = 60
    try:
        ref = []
        for xi, si in zip(x, so):
            X, s = mp.mpf(float(xi)), mp.mpf(float(si))
            h, t = X / s, s / 2
            erfcx = lambda z: mp.erfc(z) * mp.exp(z * z)
            ref.append(float(mp.sqrt(mp.pi / 2) * (erfcx(-(h + t) / mp.sqrt(2)) -
                                                   erfcx((t - h) / mp.sqrt(2)))))
    finally:
        mp.mp.dps = 15
    np.testing.assert_allclose(e[:, 0], np.array(ref), rtol=1e-12)


def test_iv_grad_at_given_sigma(orc):
    """The gradient formula at an arbitrary sigma: d sigma/dP vega(sigma) = 1;
    -d sigma/dX vega(sigma) = dP/dX at fixed sigma from central differences
    of the pinned price; at the root it is the root's gradient."""
    rng = np.random.default_rng(141)
    for model in MODELS:
        S, K, T, r, q, sig, flag = _rand_quotes(rng, 100, model, zmax=2.5)
        g = orc.iv_grad_at(model, S, K, T, r, q, sig, flag)
        vega = orc.greeks(model, S, K, T, r, q, sig, flag)["vega"]
        np.testing.assert_allclose(g[:, 0] * vega, 1.0, rtol=1e-12)

        def price(**kw):
            a = dict(fs=S, K=K, T=T, r=r, q=q)
            a.update(kw)
            hi, lo = orc.price(model, a["fs"], a["K"], a["T"], a["r"], a["q"], sig, flag,
                               with_residual=True)
            return hi.astype(np.longdouble) + lo

        names = ("fs", "K", "T", "r", "q") if model == "bsm" else ("fs", "K", "T", "r")
        for j, name in enumerate(names, 1):
            x = dict(fs=S, K=K, T=T, r=r, q=q)[name]
            h = 1e-7 * (np.abs(x) if name in ("fs", "K", "T") else np.ones_like(x))
            dP = ((price(**{name: x + h}) - price(**{name: x - h})) / (2 * h)).astype(float)
            np.testing.assert_allclose(-g[:, j] * vega, dP, rtol=1e-6, atol=1e-9, err_msg=name)
        P = orc.price(model, S, K, T, r, q, sig, flag)
        so, st = orc.implied_vol(model, P, S, K, T, r, q, flag)
        np.testing.assert_allclose(orc.iv_grad_at(model, S, K, T, r, q, so, flag),
                                   orc.iv_grad(model, P, S, K, T, r, q, flag), rtol=1e-13)
        assert np.all(np.isnan(orc.iv_grad_at(model, S[:3], K[:3], T[:3], r[:3], q[:3],
                                              np.array([0.0, -1.0, np.nan]), flag[:3])))
