"""MI355X-native batched European-option implied volatility.

Black-76 / Black-Scholes / Black-Scholes-Merton pricing, implied volatility
("Let's Be Rational" and Halley solvers), Greeks, the implicit-function IV
adjoint and ragged option chains, all computed by hand-written gfx950 HIP
kernels behind the C ABI of ``include/fastvol.h``.

The native library is loaded lazily, on the first call that needs it.
"""
from . import _native  # noqa: F401

__all__ = ["price", "implied_vol", "implied_vol_f32", "greeks", "implied_vol_backward", "implied_vol_chains",
           "price_backward", "price_autograd", "lbr_trace", "halley_trace",
           "set_halley_steps", "get_halley_steps", "normalised_black", "set_launch", "get_launch", "autotune", "version",
           "autotune_all", "launch_shape", "save_tuning", "load_tuning", "reset_tuning",
           "IVFunction", "implied_vol_autograd"]


def __getattr__(name):
    if name in ("price", "implied_vol", "implied_vol_f32", "greeks", "implied_vol_backward", "implied_vol_chains",
                "normalised_black", "set_launch", "get_launch", "autotune", "version",
                "autotune_all", "launch_shape", "save_tuning", "load_tuning", "reset_tuning",
                "price_backward", "lbr_trace", "halley_trace", "set_halley_steps",
                "get_halley_steps"):
        from . import api
        return getattr(api, name)
    if name in ("IVFunction", "implied_vol_autograd", "PriceFunction", "price_autograd"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
