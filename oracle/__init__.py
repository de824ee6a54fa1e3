"""Test-infrastructure oracle (binary128 C, OpenMP) -- NOT part of the product.

Plain, slow, scalar reference implementations of what the GPU library
computes: textbook Black-76 / Black-Scholes / Black-Scholes-Merton prices and
Greeks, the implied volatility as the exact root of the price equation, its
implicit-function gradient and the normalised Black function.  See
``fv_oracle.c`` for the definitions and their citations.

Only the test-suite, the smoke check and the CPU-baseline timing may import
this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fv_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
# FV_ORACLE_LIB names another build of the oracle to load instead (the
# mutation test points the pins at deliberately broken copies this way)
_LIB_PATH = os.environ.get("FV_ORACLE_LIB") or os.path.join(_OUT_DIR, "libfv_oracle.so")

MODELS = {"black76": 0, "bs": 1, "bsm": 2}
# status numbering of the oracle (mirrors the documented per-quote codes)
ST_OK, ST_AT, ST_BELOW, ST_ABOVE, ST_INVALID, ST_NO_EXACT_ROOT, ST_ROOT_CAP = 0, 1, 2, 3, 4, 8, 9

_lib = None


def build(force: bool = True, src: str = _SRC, out: str = None) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction); `src`
    and `out` default to fv_oracle.c and the library this module loads."""
    out = out or _LIB_PATH
    if not force and os.path.exists(out):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
           "-fPIC", src, "-o", tmp, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _model(m) -> int:
    return MODELS[m] if isinstance(m, str) else int(m)


def _bcast(n, *arrs, dtype=np.float64):
    out = []
    for a in arrs:
        a = np.asarray(a, dtype=dtype)
        out.append(np.ascontiguousarray(np.broadcast_to(a, (n,))))
    return out


def _flags(flag, n):
    f = np.asarray(flag)
    if f.dtype.kind in "US":
        f = np.where(np.char.lower(f.astype(str)) == "c", 1, -1)
    return np.ascontiguousarray(np.broadcast_to(f.astype(np.int8), (n,)))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _n(*arrs):
    shape = np.broadcast_shapes(*[np.shape(a) for a in arrs])
    return int(np.prod(shape)) if shape else 1


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    _load().orc_set_threads(ctypes.c_int(int(n)))


def price(model, fs, K, T, r, q, sigma, flag, with_residual=False):
    """Textbook price (binary128 rounded to double); optionally the residual."""
    n = _n(fs, K, T, r, q, sigma, flag)
    fs, K, T, r, q, sigma = _bcast(n, fs, K, T, r, q, sigma)
    fl = _flags(flag, n)
    hi = np.empty(n); lo = np.empty(n)
    _load().orc_price_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(fs), _p(K), _p(T),
                        _p(r), _p(q), _p(sigma), _p(fl), _p(hi), _p(lo))
    return (hi, lo) if with_residual else hi


def greeks(model, fs, K, T, r, q, sigma, flag):
    """Raw per-unit delta, gamma, vega, theta (= -dP/dT), rho."""
    n = _n(fs, K, T, r, q, sigma, flag)
    fs, K, T, r, q, sigma = _bcast(n, fs, K, T, r, q, sigma)
    fl = _flags(flag, n)
    outs = [np.empty(n) for _ in range(5)]
    _load().orc_greeks_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(fs), _p(K), _p(T),
                         _p(r), _p(q), _p(sigma), _p(fl), *[_p(o) for o in outs])
    return dict(zip(("delta", "gamma", "vega", "theta", "rho"), outs))


def status(model, price_, fs, K, T, r, q, flag):
    n = _n(price_, fs, K, T, r, q, flag)
    price_, fs, K, T, r, q = _bcast(n, price_, fs, K, T, r, q)
    fl = _flags(flag, n)
    st = np.empty(n, dtype=np.uint8)
    _load().orc_status_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(price_), _p(fs),
                         _p(K), _p(T), _p(r), _p(q), _p(fl), _p(st))
    return st


def implied_vol(model, price_, fs, K, T, r, q, flag, with_residual=False):
    """Exact root of price(sigma) = price_, rounded to double, and the status."""
    n = _n(price_, fs, K, T, r, q, flag)
    price_, fs, K, T, r, q = _bcast(n, price_, fs, K, T, r, q)
    fl = _flags(flag, n)
    sig = np.empty(n); lo = np.empty(n); st = np.empty(n, dtype=np.uint8)
    _load().orc_implied_vol_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(price_),
                              _p(fs), _p(K), _p(T), _p(r), _p(q), _p(fl), _p(sig), _p(lo),
                              _p(st))
    return (sig, lo, st) if with_residual else (sig, st)


def iv_grad(model, price_, fs, K, T, r, q, flag):
    """d sigma / d (price, S-or-F, K, T, r, q), shape (n, 6)."""
    n = _n(price_, fs, K, T, r, q, flag)
    price_, fs, K, T, r, q = _bcast(n, price_, fs, K, T, r, q)
    fl = _flags(flag, n)
    g = np.empty((n, 6))
    _load().orc_iv_grad_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(price_), _p(fs),
                          _p(K), _p(T), _p(r), _p(q), _p(fl), _p(g))
    return g


def iv_rel_sens(model, price_, fs, K, T, r, q, flag):
    """Signed relative sensitivities X d sigma/d X over X in (price, S-or-F,
    K, T, r, q) at the exact root, shape (n, 6), formed in binary128 (finite
    also where vega is far below the binary64 range)."""
    n = _n(price_, fs, K, T, r, q, flag)
    price_, fs, K, T, r, q = _bcast(n, price_, fs, K, T, r, q)
    fl = _flags(flag, n)
    e = np.empty((n, 6))
    _load().orc_iv_rel_sens_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(price_),
                              _p(fs), _p(K), _p(T), _p(r), _p(q), _p(fl), _p(e))
    return e


def iv_grad_at(model, fs, K, T, r, q, sigma, flag):
    """The implicit-function gradient d sigma/d (price, S-or-F, K, T, r, q)
    evaluated at the given sigma (not at the root), shape (n, 6)."""
    n = _n(fs, K, T, r, q, sigma, flag)
    fs, K, T, r, q, sigma = _bcast(n, fs, K, T, r, q, sigma)
    fl = _flags(flag, n)
    g = np.empty((n, 6))
    _load().orc_iv_grad_at_n(ctypes.c_int(_model(model)), ctypes.c_int64(n), _p(fs), _p(K),
                             _p(T), _p(r), _p(q), _p(sigma), _p(fl), _p(g))
    return g


def normalised_black(x, s, flag=1, with_residual=False):
    n = _n(x, s, flag)
    x, s = _bcast(n, x, s)
    fl = _flags(flag, n)
    hi = np.empty(n); lo = np.empty(n)
    _load().orc_normalised_black_n(ctypes.c_int64(n), _p(x), _p(s), _p(fl), _p(hi), _p(lo))
    return (hi, lo) if with_residual else hi
