"""Python surface of the library: thin marshalling over the C ABI.

Every argument that is a per-quote field may be a Python float (broadcast to
all quotes) or a contiguous float64 tensor on the GPU.  Results are float64
tensors on the same device, produced on the current torch stream.  Nothing
here computes: a missing or unloadable library raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

from . import _native as N


def _model(model) -> int:
    if isinstance(model, str):
        return N.MODELS[model.lower()]
    return int(model)


def _solver(solver) -> int:
    if isinstance(solver, str):
        return N.SOLVERS[solver.lower()]
    return int(solver)


# the current stream's raw handle without building a Stream object (about
# 3 us per call saved on the small-batch path)
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_ptr(stream=None, device: Optional[int] = None) -> int:
    """Raw hipStream_t of `stream`, or of torch's current stream on `device`
    (an ordinal; the current device when None)."""
    if stream is not None:
        return int(stream.cuda_stream)
    if _raw_stream is not None:
        return _raw_stream(torch.cuda.current_device() if device is None else device)
    return int(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t: torch.Tensor, name: str, dtype=torch.float64) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU (got %s)" % (name, t.device))
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _flag_arg(flag, n, keep):
    """(pointer, broadcast value) of a flag argument: 'c'/'p', +1/-1, or an
    int8 GPU tensor of n entries (kept alive in `keep`)."""
    if isinstance(flag, str):
        return None, (1 if flag.lower().startswith("c") else -1)
    if isinstance(flag, (int, float)):
        return None, int(flag)
    if isinstance(flag, torch.Tensor) and flag.dim() > 0:
        if flag.dtype != torch.int8:
            raise TypeError("flag tensor must be int8 (+1 call / -1 put)")
        _dev_tensor(flag, "flag", torch.int8)
        if flag.numel() != n:
            raise ValueError("flag length mismatch")
        keep.append(flag)
        return ctypes.c_void_p(flag.data_ptr()), 1
    raise TypeError("flag must be 'c'/'p', +1/-1 or an int8 GPU tensor")


class _Batch:
    """Validates the per-quote fields of one call in a single pass (each
    tensor: 1-D, on the GPU, float64, contiguous, one common length), and
    turns each into its fv_arg (device pointer, or broadcast value)."""

    __slots__ = ("n", "device", "args")

    def __init__(self, **fields):
        n = None
        device = None
        args = {}
        for name, v in fields.items():
            if name == "flag":
                continue
            if v is None:
                args[name] = _NO_ARG
            elif isinstance(v, torch.Tensor) and v.dim() > 0:
                if v.dim() != 1:
                    raise ValueError("%s must be 1-D" % name)
                _dev_tensor(v, name)
                m = v.numel()
                if n is None:
                    n, device = m, v.get_device()
                elif m != n:
                    raise ValueError("length mismatch: %s has %d, expected %d" % (name, m, n))
                args[name] = N.FvArg(v.data_ptr(), 0.0)
            else:
                args[name] = N.FvArg(None, float(v))
        if n is None:
            raise ValueError("at least one per-quote field must be a 1-D GPU tensor")
        self.n, self.device, self.args = n, device, args

    def arg(self, v, name) -> N.FvArg:
        a = self.args.get(name)
        if a is not None:
            return a
        # a field that was not part of the batch's construction
        if v is None:
            return _NO_ARG
        if isinstance(v, torch.Tensor) and v.dim() > 0:
            _dev_tensor(v, name)
            if v.numel() != self.n:
                raise ValueError("length mismatch: %s has %d, expected %d"
                                 % (name, v.numel(), self.n))
            return N.FvArg(v.data_ptr(), 0.0)
        return N.FvArg(None, float(v))

    def flag(self, flag):
        """Returns (pointer, broadcast value)."""
        return _flag_arg(flag, self.n, [])

    def quotes(self, price=None, fs=None, K=None, T=None, r=None, q=None, flag=1) -> N.FvQuotes:
        fp, fv = self.flag(flag)
        return N.FvQuotes(self.n, self.arg(price, "price"), self.arg(fs, "fs"), self.arg(K, "K"),
                          self.arg(T, "T"), self.arg(r, "r"),
                          self.arg(q, "q") if q is not None else _ZERO_ARG, fp, fv)

    def empty(self, dtype=torch.float64):
        return torch.empty(self.n, dtype=dtype, device=self.device)

    def rows(self, names):
        """One [len(names), n] float64 allocation, returned as a dict of its
        rows (each contiguous)."""
        block = torch.empty((len(names), self.n), dtype=torch.float64, device=self.device)
        return {k: block[i] for i, k in enumerate(names)}

    def stream(self, stream=None) -> ctypes.c_void_p:
        return ctypes.c_void_p(_stream_ptr(stream, self.device))


_NO_ARG = N.FvArg(None, 0.0)
_ZERO_ARG = N.FvArg(None, 0.0)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def price(model, fs, K, T, r, sigma, flag="c", q=None, out=None, stream=None) -> torch.Tensor:
    """Model price (Black-76: discounted, on forward fs; else spot fs)."""
    b = _Batch(fs=fs, K=K, T=T, r=r, q=q, sigma=sigma, flag=flag)
    qs = b.quotes(None, fs, K, T, r, q, flag)
    out = b.empty() if out is None else _dev_tensor(out, "out")
    N.check(N.load().fv_price(_model(model), ctypes.byref(qs), b.arg(sigma, "sigma"),
                              _ptr(out), b.stream(stream)), "fv_price")
    return out


GREEK_NAMES = ("delta", "gamma", "vega", "theta", "rho")


def _implied_vol(model, price, fs, K, T, r, flag, q, solver, greeks, with_status, stream):
    """(sigma, status or None, Greeks as one [5, n] tensor or None)."""
    b = _Batch(price=price, fs=fs, K=K, T=T, r=r, q=q, flag=flag)
    qs = b.quotes(price, fs, K, T, r, q, flag)
    sig = b.empty()
    st = b.empty(torch.uint8) if with_status else None
    G = None
    garr = None
    if greeks:
        G = torch.empty((5, b.n), dtype=torch.float64, device=b.device)
        garr = (ctypes.c_void_p * 5)(*[G[i].data_ptr() for i in range(5)])
    N.check(N.load().fv_implied_vol(_model(model), _solver(solver), ctypes.byref(qs), _ptr(sig),
                                    _ptr(st), garr, b.stream(stream)),
            "fv_implied_vol")
    return sig, st, G


def implied_vol(model, price, fs, K, T, r, flag="c", q=None, solver="lbr", greeks=False,
                with_status=True, stream=None):
    """Implied volatility.  Returns sigma, or (sigma, status) with
    ``with_status``; with ``greeks=True`` a dict of the five Greeks at the
    solved sigma is appended (rows of one [5, n] tensor)."""
    sig, st, G = _implied_vol(model, price, fs, K, T, r, flag, q, solver, greeks, with_status,
                              stream)
    res = [sig]
    if with_status:
        res.append(st)
    if greeks:
        res.append({k: G[i] for i, k in enumerate(GREEK_NAMES)})
    return res[0] if len(res) == 1 else tuple(res)


def implied_vol_f32(model, price, fs, K, T, r, flag="c", q=None, with_status=True, stream=None):
    """Implied volatility in binary32 arithmetic (Halley path): per-quote
    fields are Python floats or contiguous float32 GPU tensors; returns a
    float32 sigma (and the uint8 status with ``with_status``)."""
    fields = dict(price=price, fs=fs, K=K, T=T, r=r, q=q)
    n, device, keep = None, None, []
    for name, v in fields.items():
        if isinstance(v, torch.Tensor) and v.dim() > 0:
            _dev_tensor(v, name, torch.float32)
            if v.dim() != 1:
                raise ValueError("%s must be 1-D" % name)
            if n is None:
                n, device = v.numel(), v.device
            elif v.numel() != n:
                raise ValueError("length mismatch: %s has %d, expected %d" % (name, v.numel(), n))
    if n is None:
        raise ValueError("at least one per-quote field must be a 1-D GPU tensor")

    def arg(v, name):
        if v is None:
            return N.FvArgF32(None, 0.0)
        if isinstance(v, torch.Tensor) and v.dim() > 0:
            keep.append(v)
            return N.FvArgF32(ctypes.c_void_p(v.data_ptr()), 0.0)
        return N.FvArgF32(None, float(v))

    fp, fv = _flag_arg(flag, n, keep)
    qs = N.FvQuotesF32(n, arg(price, "price"), arg(fs, "fs"), arg(K, "K"), arg(T, "T"),
                       arg(r, "r"), arg(q if q is not None else 0.0, "q"), fp, fv)
    sig = torch.empty(n, dtype=torch.float32, device=device)
    st = torch.empty(n, dtype=torch.uint8, device=device) if with_status else None
    N.check(N.load().fv_implied_vol_f32(_model(model), ctypes.byref(qs), _ptr(sig), _ptr(st),
                                        ctypes.c_void_p(_stream_ptr(stream, sig.get_device()))),
            "fv_implied_vol_f32")
    return (sig, st) if with_status else sig


def greeks(model, fs, K, T, r, sigma, flag="c", q=None, stream=None) -> dict:
    """delta, gamma, vega, theta (= -dP/dT), rho as raw per-unit derivatives."""
    b = _Batch(fs=fs, K=K, T=T, r=r, q=q, sigma=sigma, flag=flag)
    qs = b.quotes(None, fs, K, T, r, q, flag)
    out = b.rows(("delta", "gamma", "vega", "theta", "rho"))
    N.check(N.load().fv_greeks(_model(model), ctypes.byref(qs), b.arg(sigma, "sigma"),
                               *[_ptr(v) for v in out.values()],
                               b.stream(stream)), "fv_greeks")
    return out


def implied_vol_backward(model, price, fs, K, T, r, sigma, grad_sigma, flag="c", q=None,
                         stream=None) -> dict:
    """dL/d(price, fs, K, T, r, q) from dL/dsigma (implicit-function adjoint)."""
    b = _Batch(price=price, fs=fs, K=K, T=T, r=r, q=q, flag=flag, sigma=sigma)
    qs = b.quotes(price, fs, K, T, r, q, flag)
    _dev_tensor(sigma, "sigma")
    _dev_tensor(grad_sigma, "grad_sigma")
    out = b.rows(("price", "fs", "K", "T", "r", "q"))
    N.check(N.load().fv_implied_vol_backward(_model(model), ctypes.byref(qs), _ptr(sigma),
                                             _ptr(grad_sigma), *[_ptr(v) for v in out.values()],
                                             b.stream(stream)),
            "fv_implied_vol_backward")
    return out


def price_backward(model, fs, K, T, r, sigma, grad_price, flag="c", q=None, stream=None) -> dict:
    """dL/d(fs, K, T, r, q, sigma) from dL/dprice (adjoint of ``price``)."""
    b = _Batch(fs=fs, K=K, T=T, r=r, q=q, sigma=sigma, flag=flag, grad_price=grad_price)
    qs = b.quotes(None, fs, K, T, r, q, flag)
    _dev_tensor(grad_price, "grad_price")
    out = b.rows(("fs", "K", "T", "r", "q", "sigma"))
    N.check(N.load().fv_price_backward(_model(model), ctypes.byref(qs), b.arg(sigma, "sigma"),
                                       _ptr(grad_price), *[_ptr(v) for v in out.values()],
                                       b.stream(stream)), "fv_price_backward")
    return out


def implied_vol_chains(chain_mat_off, mat_quote_off, F, r, T, price, K, flag, solver="lbr",
                       with_status=True, stream=None):
    """Implied volatility of ragged Black-76 chains (CSR offsets, int64)."""
    for t, nm in ((chain_mat_off, "chain_mat_off"), (mat_quote_off, "mat_quote_off")):
        _dev_tensor(t, nm, torch.int64)
    for t, nm in ((F, "F"), (r, "r"), (T, "T"), (price, "price"), (K, "K")):
        _dev_tensor(t, nm)
    _dev_tensor(flag, "flag", torch.int8)
    c = N.FvChains(F.numel(), T.numel(), price.numel(), _ptr(chain_mat_off), _ptr(mat_quote_off),
                   _ptr(F), _ptr(r), _ptr(T), _ptr(price), _ptr(K), _ptr(flag))
    if chain_mat_off.numel() != F.numel() + 1 or mat_quote_off.numel() != T.numel() + 1:
        raise ValueError("offset arrays must have n_chains+1 and n_maturities+1 entries")
    if K.numel() != price.numel() or flag.numel() != price.numel() or r.numel() != F.numel():
        raise ValueError("per-quote / per-chain array lengths disagree")
    sig = torch.empty(price.numel(), dtype=torch.float64, device=price.device)
    st = torch.empty(price.numel(), dtype=torch.uint8, device=price.device) if with_status else None
    N.check(N.load().fv_implied_vol_chains(_solver(solver), ctypes.byref(c), _ptr(sig), _ptr(st),
                                           ctypes.c_void_p(_stream_ptr(stream, sig.get_device()))),
            "fv_implied_vol_chains")
    return (sig, st) if with_status else sig


def normalised_black(x, s, flag=None, stream=None) -> torch.Tensor:
    _dev_tensor(x, "x")
    _dev_tensor(s, "s")
    if flag is not None:
        _dev_tensor(flag, "flag", torch.int8)
    if x.numel() != s.numel():
        raise ValueError("x and s lengths differ")
    out = torch.empty_like(x)
    N.check(N.load().fv_normalised_black(x.numel(), _ptr(x), _ptr(s), _ptr(flag), _ptr(out),
                                         ctypes.c_void_p(_stream_ptr(stream, out.get_device()))),
            "fv_normalised_black")
    return out


def lbr_trace(model, price, fs, K, T, r, flag="c", q=None, stream=None) -> torch.Tensor:
    """Per-quote path code of the LBR solver (see fv_lbr_trace)."""
    b = _Batch(price=price, fs=fs, K=K, T=T, r=r, q=q, flag=flag)
    qs = b.quotes(price, fs, K, T, r, q, flag)
    out = torch.empty(b.n, dtype=torch.int32, device=b.device)
    N.check(N.load().fv_lbr_trace(_model(model), ctypes.byref(qs), _ptr(out),
                                  b.stream(stream)), "fv_lbr_trace")
    return out


def halley_trace(model, price, fs, K, T, r, flag="c", q=None, stream=None) -> torch.Tensor:
    """Per-quote Halley step count and fallback bit (see fv_halley_trace)."""
    b = _Batch(price=price, fs=fs, K=K, T=T, r=r, q=q, flag=flag)
    qs = b.quotes(price, fs, K, T, r, q, flag)
    out = torch.empty(b.n, dtype=torch.int32, device=b.device)
    N.check(N.load().fv_halley_trace(_model(model), ctypes.byref(qs), _ptr(out),
                                     b.stream(stream)), "fv_halley_trace")
    return out


def set_halley_steps(steps: int) -> None:
    """Halley steps before the bisection fallback (fv_set_halley_steps)."""
    N.check(N.load().fv_set_halley_steps(int(steps)), "fv_set_halley_steps")


def get_halley_steps() -> int:
    return int(N.load().fv_get_halley_steps())


def set_launch(kernel, block: int, quotes_per_thread: int) -> None:
    k = N.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    N.check(N.load().fv_set_launch(k, int(block), int(quotes_per_thread)), "fv_set_launch")


def get_launch(kernel):
    k = N.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    b, q = ctypes.c_int(), ctypes.c_int()
    N.check(N.load().fv_get_launch(k, ctypes.byref(b), ctypes.byref(q)), "fv_get_launch")
    return b.value, q.value


def autotune(kernel, model="bsm", n_hint: int = 1 << 22, stream=None):
    """Time the launch shapes of one kernel family on `n_hint` synthetic
    quotes and keep the fastest for that model and size class; returns it."""
    k = N.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    N.check(N.load().fv_autotune(k, _model(model), int(n_hint),
                                 ctypes.c_void_p(_stream_ptr(stream))), "fv_autotune")
    return launch_shape(k, model, max(1, int(n_hint)))


# one batch size per size class of the tuning table (2^12 .. 2^24)
TUNING_SIZES = (1 << 12, 1 << 15, 1 << 17, 1 << 19, 1 << 21, 1 << 23, 1 << 24)


def autotune_all(kernels=None, models=("bsm",), sizes=TUNING_SIZES, stream=None) -> dict:
    """fv_autotune over kernel families x models x sizes; returns
    {(kernel, model, size): (block, quotes_per_thread)}."""
    kernels = kernels or [k for k in N.KERNELS]
    out = {}
    for kern in kernels:
        for model in (("black76",) if kern == "chains" else models):
            for n in sizes:
                out[(kern, model, n)] = autotune(kern, model, n, stream)
    return out


def launch_shape(kernel, model, n: int):
    """(block, quotes per thread) a launch of n quotes would use."""
    k = N.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    b, q = ctypes.c_int(), ctypes.c_int()
    N.check(N.load().fv_launch_shape(k, _model(model), int(n), ctypes.byref(b), ctypes.byref(q)),
            "fv_launch_shape")
    return b.value, q.value


def save_tuning(path) -> None:
    N.check(N.load().fv_tuning_save(os.fsencode(path)), "fv_tuning_save")


def load_tuning(path) -> None:
    N.check(N.load().fv_tuning_load(os.fsencode(path)), "fv_tuning_load")


def reset_tuning() -> None:
    N.check(N.load().fv_tuning_reset(), "fv_tuning_reset")


def version() -> int:
    return int(N.load().fv_version())
