"""Differentiable implied volatility and pricing (the paper's section 3,
"Differentiable IV": an autograd-friendly implied-volatility entry point).

IVFunction: forward is one fv_implied_vol launch; backward is one
fv_implied_vol_backward launch, the implicit-function adjoint
    dsigma/dP = 1/vega,  dsigma/dX = -(dP/dX at fixed sigma)/vega,
so no iteration is unrolled or differentiated.

PriceFunction: forward fv_price, backward from fv_greeks (vega, delta,
theta, rho) and the strike / dividend partials -- it lets a loss flow
through "volatility -> price -> implied volatility" (e.g. calibration).
"""
from __future__ import annotations

import torch

from . import api


def _req(t):
    return isinstance(t, torch.Tensor) and t.requires_grad


class IVFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, price, fs, K, T, r, q, flag, model, solver, greeks):
        sig, st, G = api._implied_vol(model, price.detach(), _d(fs), _d(K), _d(T), _d(r), flag,
                                      _d(q), solver, greeks, True, None)
        ctx.model = model
        ctx.flag = flag
        ctx.scalar = [not isinstance(v, torch.Tensor) or v.dim() == 0 for v in (price, fs, K, T, r, q)]
        ctx.save_for_backward(*[v if isinstance(v, torch.Tensor) else torch.tensor(float(v or 0.0))
                                for v in (price, fs, K, T, r, q)], sig)
        # the five Greeks leave as one [5, n] tensor: every extra output of a
        # Function costs the autograd engine bookkeeping
        extra = (G,) if greeks else ()
        ctx.mark_non_differentiable(st, *extra)
        return (sig, st) + extra

    @staticmethod
    def backward(ctx, g_sig, g_st, *g_greeks):
        price, fs, K, T, r, q, sig = ctx.saved_tensors
        args = [v.item() if s else v.detach() for v, s in zip((price, fs, K, T, r, q), ctx.scalar)]
        g = api.implied_vol_backward(ctx.model, args[0], args[1], args[2], args[3], args[4],
                                     sig, g_sig.contiguous(), flag=ctx.flag, q=args[5])
        return (*_input_grads(g, ("price", "fs", "K", "T", "r", "q"), ctx.scalar,
                              ctx.needs_input_grad[:6], (price, fs, K, T, r, q)),
                None, None, None, None)


def _d(v):
    return v.detach() if isinstance(v, torch.Tensor) else v


def _input_grads(g, names, scalar, needs, saved):
    """Gradient of each input from the per-quote adjoint rows g[name]: the row
    itself for a per-quote tensor; for a 0-dim tensor broadcast to every
    quote (a shared r or T, say) the sum of the row over the quotes, with the
    input's dtype and device; None where no gradient is needed."""
    outs = []
    for name, s, need, v in zip(names, scalar, needs, saved):
        if not need:
            outs.append(None)
        elif s:
            outs.append(g[name].sum().to(dtype=v.dtype, device=v.device).reshape(v.shape))
        else:
            outs.append(g[name])
    return outs


def implied_vol_autograd(model, price, fs, K, T, r, flag="c", q=None, solver="lbr",
                         greeks=False):
    """Implied volatility with gradients to every tensor input.  Returns
    (sigma, status), or (sigma, status, greeks) with ``greeks=True``: the
    five Greeks at the solved sigma from the same fused launch, as a dict
    (delta, gamma, vega, theta, rho).  Status and Greeks are not
    differentiable."""
    out = IVFunction.apply(price, fs, K, T, r, q, flag, model, solver, bool(greeks))
    if not greeks:
        return out
    return out[0], out[1], {k: out[2][i] for i, k in enumerate(api.GREEK_NAMES)}


class PriceFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fs, K, T, r, q, sigma, flag, model):
        p = api.price(model, _d(fs), _d(K), _d(T), _d(r), _d(sigma), flag=flag, q=_d(q))
        ctx.model, ctx.flag = model, flag
        ctx.scalar = [not isinstance(v, torch.Tensor) or v.dim() == 0 for v in (fs, K, T, r, q, sigma)]
        ctx.save_for_backward(*[v if isinstance(v, torch.Tensor) else torch.tensor(float(v or 0.0))
                                for v in (fs, K, T, r, q, sigma)])
        return p

    @staticmethod
    def backward(ctx, g_p):
        saved = ctx.saved_tensors
        a = [v.item() if s else v.detach() for v, s in zip(saved, ctx.scalar)]
        g = api.price_backward(ctx.model, a[0], a[1], a[2], a[3], a[5], g_p.contiguous(),
                               flag=ctx.flag, q=a[4])
        return (*_input_grads(g, ("fs", "K", "T", "r", "q", "sigma"), ctx.scalar,
                              ctx.needs_input_grad[:6], saved), None, None)


def price_autograd(model, fs, K, T, r, sigma, flag="c", q=None):
    return PriceFunction.apply(fs, K, T, r, q, sigma, flag, model)
