"""py_vollib-style calling surface over the library (the public API the paper
lists in its "Capabilities" section and Table of entry points).

Names and argument orders follow the paper:
  fast_black(flag, F, K, t, r, sigma)                     Black-76 (discounted)
  fast_black_scholes(flag, S, K, t, r, sigma)
  fast_black_scholes_merton(flag, S, K, t, r, sigma, q)
  fast_implied_volatility(price, S, K, t, r, flag, q=None)        BS / BSM
  fast_implied_volatility_black(mid, F, K, r, T, flag)    note: r before T;
      `mid` is the discounted Black-76 price and the same r discounts and
      inverts (paper section "Black-76 Convention")
  vectorized_{delta,gamma,theta,rho,vega}(flag, S, K, t, r, sigma, q=None,
      model="black_scholes")
  get_all_greeks(flag, S, K, t, r, sigma, q=None, model="black_scholes")

Inputs are array-likes (scalars, lists, numpy arrays, torch tensors)
broadcast with numpy's rules; flags are "c"/"p" (a string or an array of
strings) or +1/-1.  Results have the broadcast shape and are numpy arrays
(``return_as="numpy"``) or float64 GPU tensors (``return_as="torch"``).

The IV entry points use the Halley solver by default, as the paper's public
API does; ``solver="lbr"`` selects "Let's Be Rational".  Quotes whose price
has no implied volatility return NaN (0 exactly at the intrinsic value).

Greeks are scaled as py_vollib reports them unless ``scaling="raw"``:
theta per calendar day (the per-year theta / 365), vega and rho per
percentage point (/ 100); delta and gamma per unit.  This reading of
py_vollib's units is not checked against py_vollib here (it is not
installed); ``scaling="raw"`` returns the library's per-unit derivatives.

Everything is computed by the library's kernels; this module only converts
and broadcasts arguments (and applies the constant unit factors above).
"""
from __future__ import annotations

import numpy as np
import torch

from . import api

_MODELS = {"black": "black76", "black76": "black76", "black_scholes": "bs", "bs": "bs",
           "black_scholes_merton": "bsm", "bsm": "bsm"}


def _is_scalar(v) -> bool:
    if isinstance(v, torch.Tensor):
        return v.dim() == 0
    return np.ndim(v) == 0


def _flag_array(flag):
    """int8 numpy array (or python int) from "c"/"p" strings or +-1."""
    if isinstance(flag, torch.Tensor):
        flag = flag.detach().cpu().numpy()
    if isinstance(flag, str):
        return 1 if flag.lower().startswith("c") else -1
    a = np.asarray(flag)
    if a.dtype.kind in ("U", "S", "O"):
        low = np.char.lower(a.astype(str))
        if not np.all(np.char.startswith(low, "c") | np.char.startswith(low, "p")):
            raise ValueError("flags must be 'c' or 'p'")
        out = np.where(np.char.startswith(low, "c"), 1, -1).astype(np.int8)
    else:
        if not np.all(np.isin(a, (1, -1))):
            raise ValueError("numeric flags must be +1 (call) or -1 (put)")
        out = a.astype(np.int8)
    return int(out) if out.ndim == 0 else out


def _prepare(fields: dict, flag):
    """Broadcast the numeric fields and the flag; returns (shape, converted
    fields, converted flag).  Scalars stay Python floats (broadcast by the
    library); arrays become flat float64 GPU tensors of the broadcast shape."""
    fl = _flag_array(flag)
    shapes = [tuple(v.shape) if isinstance(v, torch.Tensor) else np.shape(v)
              for v in fields.values() if v is not None]
    if not isinstance(fl, int):
        shapes.append(fl.shape)
    shape = np.broadcast_shapes(*shapes) if shapes else ()
    n = int(np.prod(shape)) if shape else 1
    out = {}
    for name, v in fields.items():
        if v is None:
            out[name] = None
        elif _is_scalar(v):
            out[name] = float(v.item() if isinstance(v, torch.Tensor) else v)
        else:
            a = v.detach().to("cpu", torch.float64).numpy() if isinstance(v, torch.Tensor) \
                else np.asarray(v, dtype=np.float64)
            # a writable copy: broadcast views are read-only
            a = np.array(np.broadcast_to(a, shape).reshape(-1), dtype=np.float64)
            out[name] = torch.from_numpy(a).to("cuda")
    if isinstance(fl, int):
        fl_out = fl
    else:
        f = np.array(np.broadcast_to(fl, shape).reshape(-1))
        fl_out = torch.from_numpy(f).to("cuda")
    # the library needs one per-quote array to size the batch
    if not any(isinstance(v, torch.Tensor) for v in out.values()) and \
            not isinstance(fl_out, torch.Tensor):
        key = next(k for k, v in out.items() if v is not None)
        out[key] = torch.full((n,), out[key], dtype=torch.float64, device="cuda")
    return shape, out, fl_out


def _finish(t: torch.Tensor, shape, return_as: str):
    t = t.reshape(shape) if shape else t.reshape(())
    if return_as == "torch":
        return t
    if return_as == "numpy":
        return t.cpu().numpy()
    raise ValueError("return_as must be 'numpy' or 'torch'")


def _price(model, flag, fs, K, t, r, sigma, q, return_as):
    shape, f, fl = _prepare({"fs": fs, "K": K, "T": t, "r": r, "sigma": sigma, "q": q}, flag)
    p = api.price(model, f["fs"], f["K"], f["T"], f["r"], f["sigma"], flag=fl, q=f["q"])
    return _finish(p, shape, return_as)


def fast_black(flag, F, K, t, r, sigma, return_as="numpy"):
    """Discounted Black-76 price on the forward F."""
    return _price("black76", flag, F, K, t, r, sigma, None, return_as)


def fast_black_scholes(flag, S, K, t, r, sigma, return_as="numpy"):
    return _price("bs", flag, S, K, t, r, sigma, None, return_as)


def fast_black_scholes_merton(flag, S, K, t, r, sigma, q, return_as="numpy"):
    return _price("bsm", flag, S, K, t, r, sigma, q, return_as)


def _iv(model, price, fs, K, t, r, flag, q, solver, return_as):
    shape, f, fl = _prepare({"price": price, "fs": fs, "K": K, "T": t, "r": r, "q": q}, flag)
    sig = api.implied_vol(model, f["price"], f["fs"], f["K"], f["T"], f["r"], flag=fl,
                          q=f["q"], solver=solver, with_status=False)
    return _finish(sig, shape, return_as)


def fast_implied_volatility(price, S, K, t, r, flag, q=None, solver="halley", return_as="numpy"):
    """IV of Black-Scholes (q None) or Black-Scholes-Merton prices."""
    return _iv("bs" if q is None else "bsm", price, S, K, t, r, flag, q, solver, return_as)


def fast_implied_volatility_black(mid, F, K, r, T, flag, solver="halley", return_as="numpy"):
    """IV of discounted Black-76 prices (r discounts and inverts)."""
    return _iv("black76", mid, F, K, T, r, flag, None, solver, return_as)


_SCALE = {"delta": 1.0, "gamma": 1.0, "theta": 1.0 / 365.0, "vega": 0.01, "rho": 0.01}


def get_all_greeks(flag, S, K, t, r, sigma, q=None, model="black_scholes", scaling="py_vollib",
                   return_as="numpy"):
    """delta, gamma, theta, rho, vega in one library call (dict)."""
    m = _MODELS[model]
    if m == "bsm" and q is None:
        raise ValueError("model black_scholes_merton needs q")
    shape, f, fl = _prepare({"fs": S, "K": K, "T": t, "r": r, "sigma": sigma,
                             "q": q if m == "bsm" else None}, flag)
    g = api.greeks(m, f["fs"], f["K"], f["T"], f["r"], f["sigma"], flag=fl, q=f["q"])
    if scaling not in ("py_vollib", "raw"):
        raise ValueError("scaling must be 'py_vollib' or 'raw'")
    out = {}
    for k in ("delta", "gamma", "theta", "rho", "vega"):
        v = g[k] if scaling == "raw" or _SCALE[k] == 1.0 else g[k] * _SCALE[k]
        out[k] = _finish(v, shape, return_as)
    return out


def _one(name):
    def fn(flag, S, K, t, r, sigma, q=None, model="black_scholes", scaling="py_vollib",
           return_as="numpy"):
        return get_all_greeks(flag, S, K, t, r, sigma, q, model, scaling, return_as)[name]
    fn.__name__ = "vectorized_" + name
    fn.__doc__ = "%s of every quote (see get_all_greeks for units)." % name
    return fn


vectorized_delta = _one("delta")
vectorized_gamma = _one("gamma")
vectorized_theta = _one("theta")
vectorized_rho = _one("rho")
vectorized_vega = _one("vega")

__all__ = ["fast_black", "fast_black_scholes", "fast_black_scholes_merton",
           "fast_implied_volatility", "fast_implied_volatility_black", "get_all_greeks",
           "vectorized_delta", "vectorized_gamma", "vectorized_theta", "vectorized_rho",
           "vectorized_vega"]
