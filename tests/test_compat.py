"""py_vollib-style surface: argument orders, flags, broadcasting, units."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def test_flag_parsing_cpu():
    from paper_2604_27210_amd.compat import _flag_array
    assert _flag_array("c") == 1 and _flag_array("P") == -1
    np.testing.assert_array_equal(_flag_array(np.array(["c", "p", "C"])), [1, -1, 1])
    np.testing.assert_array_equal(_flag_array([1, -1]), [1, -1])
    with pytest.raises(ValueError):
        _flag_array(np.array(["c", "x"]))
    with pytest.raises(ValueError):
        _flag_array([1, 0])


@pytest.fixture(scope="module")
def cp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_27210_amd as fv
    fv._native.load()
    from paper_2604_27210_amd import compat
    return compat


@pytest.mark.gpu
def test_minimal_example_round_trip(cp):
    """The paper's minimal example: three BS prices, then their IVs."""
    K = np.array([95.0, 100.0, 105.0])
    fl = np.array(["c", "c", "p"])
    p = cp.fast_black_scholes(fl, 100.0, K, 0.25, 0.05, 0.20)
    po = oracle.price("bs", np.full(3, 100.0), K, np.full(3, 0.25), np.full(3, 0.05), 0.0,
                      np.full(3, 0.2), np.array([1, 1, -1], dtype=np.int8))
    np.testing.assert_allclose(p, po, rtol=1e-13)
    for solver in ("halley", "lbr"):
        iv = cp.fast_implied_volatility(p, 100.0, K, 0.25, 0.05, fl, solver=solver)
        np.testing.assert_allclose(iv, 0.2, rtol=1e-8 if solver == "halley" else 1e-12)


@pytest.mark.gpu
def test_black76_argument_order_and_broadcast(cp):
    F = np.array([[90.0], [110.0]])           # (2, 1)
    K = np.array([80.0, 100.0, 120.0])        # (3,)
    mid = cp.fast_black("p", F, K, 0.5, 0.03, 0.3)
    assert mid.shape == (2, 3)
    Fb, Kb = np.broadcast_arrays(F, K)
    po = oracle.price("black76", Fb.ravel(), Kb.ravel(), np.full(6, 0.5), np.full(6, 0.03), 0.0,
                      np.full(6, 0.3), np.full(6, -1, dtype=np.int8))
    np.testing.assert_allclose(mid.ravel(), po, rtol=1e-13)
    # fast_implied_volatility_black takes (mid, F, K, r, T, flag)
    iv = cp.fast_implied_volatility_black(mid, F, K, 0.03, 0.5, "p", solver="lbr")
    np.testing.assert_allclose(iv, 0.3, rtol=1e-12)
    t = cp.fast_black("c", F, K, 0.5, 0.03, 0.3, return_as="torch")
    assert t.is_cuda and t.shape == (2, 3)


@pytest.mark.gpu
def test_merton_and_greeks_units(cp):
    rng = np.random.default_rng(7)
    n = 64
    S, K = 100.0, 100.0 * np.exp(rng.uniform(-0.3, 0.3, n))
    t, r, q, sig = rng.uniform(0.1, 2, n), 0.02, 0.01, rng.uniform(0.1, 0.6, n)
    fl = np.where(rng.random(n) < 0.5, "c", "p")
    p = cp.fast_black_scholes_merton(fl, S, K, t, r, sig, q)
    fli = np.where(fl == "c", 1, -1).astype(np.int8)
    po = oracle.price("bsm", np.full(n, S), K, t, np.full(n, r), np.full(n, q), sig, fli)
    np.testing.assert_allclose(p, po, rtol=1e-12)
    raw = cp.get_all_greeks(fl, S, K, t, r, sig, q=q, model="black_scholes_merton", scaling="raw")
    g = cp.get_all_greeks(fl, S, K, t, r, sig, q=q, model="black_scholes_merton")
    go = oracle.greeks("bsm", np.full(n, S), K, t, np.full(n, r), np.full(n, q), sig, fli)
    for k in ("delta", "gamma", "vega", "theta", "rho"):
        np.testing.assert_allclose(raw[k], go[k], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g["theta"], raw["theta"] / 365.0, rtol=1e-15)
    np.testing.assert_allclose(g["vega"], raw["vega"] / 100.0, rtol=1e-15)
    np.testing.assert_allclose(g["rho"], raw["rho"] / 100.0, rtol=1e-15)
    np.testing.assert_array_equal(g["delta"], raw["delta"])
    np.testing.assert_array_equal(cp.vectorized_vega(fl, S, K, t, r, sig, q=q,
                                                     model="black_scholes_merton"), g["vega"])


@pytest.mark.gpu
def test_all_scalar_call(cp):
    p = cp.fast_black_scholes("c", 100.0, 100.0, 1.0, 0.0, 0.2)
    assert p.shape == ()
    iv = cp.fast_implied_volatility(p, 100.0, 100.0, 1.0, 0.0, "c")
    assert abs(float(iv) - 0.2) < 1e-8
