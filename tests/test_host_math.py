"""The reduction's exponentials and log-moneyness, compiled for the host from
the kernels' own headers (g++), against mpmath (CPU only).

- e^{r T} and e^{(r - q) T} carry the rounding of their exponent: within
  4 ulps of the exact value at r T up to 40, where a rounded binary64
  exponent alone would be tens of ulps off;
- ln(F/K) stays finite and accurate where F/K leaves the binary64 range."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r'''
#include <cstdint>
#include "fv_quote.h"
extern "C" {
void h_exp_prod(int64_t n, const double* a, const double* b, double* o) {
  for (int64_t i = 0; i < n; ++i) o[i] = fv::fexp_prod(a[i], b[i]);
}
void h_exp_carry(int64_t n, const double* r, const double* q, const double* T, double* o) {
  for (int64_t i = 0; i < n; ++i) o[i] = fv::fexp_carry(r[i], q[i], T[i]);
}
// Black-76 implied volatility with either solver, as the flat kernels run
// it per quote (solver 0: LBR, 1: Halley with the bisection fallback)
void h_iv_b76(int solver, int64_t n, const double* P, const double* F, const double* K,
              const double* T, const double* r, const int* th, double* sig, int* st) {
  for (int64_t i = 0; i < n; ++i) {
    const fv::Reduced rd = fv::reduce_quote(fv::kBlack76, P[i], F[i], K[i], T[i], r[i], 0.0, th[i]);
    int s_ = rd.status;
    double sg = s_ == fv::kQAtIntrinsic ? 0.0 : __builtin_nan("");
    if (s_ == fv::kQOk) {
      if (solver == 0) {
        const fv::LbrResult res = fv::lbr_solve(rd.x, rd.beta, rd.bmax, rd.lnb, 2, 4, 1e-6);
        sg = res.s * rd.isqrtT;
        if (!res.converged) s_ = fv::kQNotConverged;
      } else {
        const fv::HalleyState hs = fv::halley_solve(rd.x, rd.beta, rd.bmax, rd.lnb, 8);
        double s = hs.s;
        if (!hs.converged) s = fv::bisection_solve(rd.x, rd.beta, rd.bmax, rd.lnb, hs.lo, hs.hi, 1e-13);
        sg = s * rd.isqrtT;
      }
    }
    sig[i] = sg;
    st[i] = s_;
  }
}
// price_at and greeks_at as the pricing, Greeks and fused kernels call them
void h_price_greeks(int64_t n, const double* F, const double* K, const double* T,
                    const double* sig, const int* th, double* price, double* greeks) {
  for (int64_t i = 0; i < n; ++i) {
    const double D = 1.0;
    price[i] = fv::price_at(F[i], K[i], D, sig[i], fv::sqrt_pos(T[i]), th[i]);
    const fv::Greeks g = fv::greeks_at(fv::kBlack76, F[i], K[i], T[i], 0.0, 0.0, sig[i], th[i],
                                       F[i], D, price[i]);
    greeks[5 * i + 0] = g.delta;
    greeks[5 * i + 1] = g.gamma;
    greeks[5 * i + 2] = g.vega;
    greeks[5 * i + 3] = g.theta;
    greeks[5 * i + 4] = g.rho;
  }
}
void h_reduce_x(int64_t n, const double* P, const double* F, const double* K, double* x,
                int* st) {
  for (int64_t i = 0; i < n; ++i) {
    const fv::Reduced rd = fv::reduce_quote(fv::kBlack76, P[i], F[i], K[i], 1.0, 0.0, 0.0, 1);
    x[i] = rd.x;
    st[i] = rd.status;
  }
}
}
'''


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostmath")
    src = d / "hm.cpp"
    src.write_text(SRC)
    so = d / "libhm.so"
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2604_27210_amd", "csrc"), str(src), "-o", str(so)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.skip("host build of the kernel headers failed: " + res.stderr[-500:])
    return ctypes.CDLL(str(so))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ulps(got, exact):
    return np.array([float(abs(mp.mpf(g) - e) / (abs(e) * mp.mpf(2) ** -52)) for g, e in zip(got, exact)])


def test_exponent_rounding_is_carried(lib):
    mp.mp.dps = 40
    rng = np.random.default_rng(5)
    n = 2000
    r = rng.uniform(-0.5, 0.5, n)
    q = rng.uniform(-0.2, 0.4, n)
    T = rng.uniform(10.0, 80.0, n)
    o = np.empty(n)
    lib.h_exp_prod(ctypes.c_int64(n), _p(r), _p(T), _p(o))
    exact = [mp.e ** (mp.mpf(a) * mp.mpf(b)) for a, b in zip(r, T)]
    assert _ulps(o, exact).max() <= 4.0
    # the naive form, for contrast: the rounded exponent alone costs tens of ulps
    naive = np.exp(r * T)
    assert _ulps(naive, exact).max() > 8.0
    lib.h_exp_carry(ctypes.c_int64(n), _p(r), _p(q), _p(T), _p(o))
    exact = [mp.e ** ((mp.mpf(a) - mp.mpf(c)) * mp.mpf(b)) for a, c, b in zip(r, q, T)]
    assert _ulps(o, exact).max() <= 4.0


def test_log_moneyness_beyond_the_ratio_range(lib):
    mp.mp.dps = 40
    # out-of-the-money calls (K > F) with F/K below the binary64 range, at its
    # edge, and an ordinary one; prices below the upper bound F
    F = np.array([1e-300, 1e-200, 1e-154, 3.0, 1e-160])
    K = np.array([1e300, 1e200, 1e154, 5.0, 1e150])
    P = np.array([1e-303, 1e-203, 1e-157, 0.1, 1e-163])
    x = np.empty(5)
    st = np.zeros(5, dtype=np.int32)
    lib.h_reduce_x(ctypes.c_int64(5), _p(P), _p(F), _p(K), _p(x), _p(st))
    for i in range(5):
        if st[i] != 0:
            continue
        lx = float(mp.log(mp.mpf(F[i]) / mp.mpf(K[i])))
        assert np.isfinite(x[i]) and abs(abs(x[i]) - abs(lx)) <= 1e-13 * abs(lx), (i, x[i], lx)
    assert (st == 0).all(), st


def _subnormal_cells():
    """Black-76 out-of-the-money calls (F = 1, K = e^{-x}, T = 1, r = 0) on
    the accuracy plane's grid whose price is below the normal binary64
    range, plus a forward and strike near the top of the range whose
    normalised price underflows to zero (ln beta = -1382.7)."""
    import oracle
    xs = np.concatenate([[0.0], -np.logspace(-4, np.log10(20.0), 159)])
    ss = np.logspace(-3, np.log10(8.0), 160)
    X, S = (a.ravel() for a in np.meshgrid(xs, ss, indexing="ij"))
    K = np.exp(-X)
    one = np.ones_like(X)
    P = oracle.price("black76", one, K, one, 0 * one, 0.0, S, 1)
    so, st = oracle.implied_vol("black76", P, one, K, one, 0 * one, 0.0, 1)
    keep = (st == 0) & (P > 0) & (P < 2.2250738585072014e-308)
    F = np.concatenate([one[keep], [1e300]])
    K = np.concatenate([K[keep], [1e301]])
    P = np.concatenate([P[keep], [1e-300]])
    return F, K, P


@pytest.mark.parametrize("solver", [0, 1])
def test_subnormal_prices_solved_or_flagged(lib, solver):
    """Prices below the normal binary64 range (the accuracy plane's 26 cells
    and a normalised price that underflows to zero): both solvers of the
    kernels' own code, compiled for the host, return the oracle's root within
    the parity tolerance (1e-12 LBR, 1e-8 Halley, or the inputs' rounding
    sensitivity) -- never a wrong sigma with status OK."""
    import oracle
    F, K, P = _subnormal_cells()
    n = len(F)
    assert n >= 20
    one = np.ones(n)
    th = np.ones(n, dtype=np.int32)
    sig = np.empty(n)
    st = np.zeros(n, dtype=np.int32)
    lib.h_iv_b76(ctypes.c_int(solver), ctypes.c_int64(n), _p(P), _p(F), _p(K), _p(one),
                 _p(0 * one), _p(th), _p(sig), _p(st))
    so, sto = oracle.implied_vol("black76", P, F, K, one, 0 * one, 0.0, 1)
    assert np.all(sto == 0)
    cabs = np.sum(np.abs(oracle.iv_rel_sens("black76", P, F, K, one, 0 * one, 0.0, 1)), 1)
    assert np.all(np.isfinite(cabs))
    base = np.maximum(1e-12 * so, 2e-13) if solver == 0 else 1e-8 * so
    tol = np.maximum(base, 8 * 2.0 ** -53 * cabs)
    assert np.all(st == 0), (solver, st)
    err = np.abs(sig - so)
    assert np.all(err <= tol), (solver, np.max(err / tol), sig[err > tol][:4], so[err > tol][:4])


def test_price_and_greeks_beyond_the_ratio_range(lib):
    """price_at and greeks_at where F/K leaves the binary64 range (the
    reduction's own log-moneyness rule), against the oracle: finite and
    within a few ulps of its condition."""
    import oracle
    F = np.array([1e-300, 1e-200, 1e300, 3.0])
    K = np.array([1e300, 1e200, 1e-300, 5.0])
    T = np.ones(4)
    sig = np.array([30.0, 20.0, 30.0, 0.3])
    th = np.array([1, -1, -1, 1], dtype=np.int32)
    price = np.empty(4)
    g = np.empty(20)
    lib.h_price_greeks(ctypes.c_int64(4), _p(F), _p(K), _p(T), _p(sig), _p(th), _p(price), _p(g))
    g = g.reshape(4, 5)
    po = oracle.price("black76", F, K, T, 0 * T, 0.0, sig, th.astype(np.int8))
    go = oracle.greeks("black76", F, K, T, 0 * T, 0.0, sig, th.astype(np.int8))
    assert np.all(np.isfinite(price)) and np.all(np.isfinite(g))
    # log-moneyness ~1400 carries ~1400 u of absolute error into d1, d2
    np.testing.assert_allclose(price, po, rtol=1e-9)
    for j, name in enumerate(("delta", "gamma", "vega", "theta", "rho")):
        np.testing.assert_allclose(g[:, j], go[name], rtol=1e-9, atol=1e-300, err_msg=name)
