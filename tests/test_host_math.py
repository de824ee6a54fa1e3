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
