"""ctypes declarations of the C ABI in ``include/fastvol.h``.

Only argument marshalling lives here: every computation happens in the
gfx950 kernels of ``libfastvol.so``.  The library is loaded after torch so
that it binds to the HIP runtime torch already mapped (same SONAME), which
makes torch device pointers and streams valid in it.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FASTVOL_LIBRARY may name another build of the same library (e.g. one
# compiled with different register-allocation targets)
LIB_PATH = os.environ.get("FASTVOL_LIBRARY") or os.path.join(HERE, "_build", "libfastvol.so")

FV_OK = 0
FV_E_INVALID_ARG = -1
FV_E_HIP = -2
FV_E_UNSUPPORTED = -3

MODELS = {"black76": 0, "black": 0, "b76": 0, "bs": 1, "black_scholes": 1, "bsm": 2,
          "black_scholes_merton": 2}
SOLVERS = {"lbr": 0, "jackel": 0, "halley": 1}
KERNELS = {"price": 0, "iv_lbr": 1, "iv_halley": 2, "greeks": 3, "backward": 4, "chains": 5,
           "iv_halley_f32": 6}

# per-quote status codes
Q_OK, Q_AT_INTRINSIC, Q_BELOW_INTRINSIC, Q_ABOVE_MAX, Q_INVALID_INPUT, Q_NOT_CONVERGED = range(6)


class FvArg(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("value", ctypes.c_double)]


class FvQuotes(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("price", FvArg), ("fs", FvArg), ("K", FvArg), ("T", FvArg), ("r", FvArg),
                ("q", FvArg),
                ("flag", ctypes.c_void_p), ("flag_value", ctypes.c_int8)]


class FvArgF32(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("value", ctypes.c_float)]


class FvQuotesF32(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("price", FvArgF32), ("fs", FvArgF32), ("K", FvArgF32), ("T", FvArgF32),
                ("r", FvArgF32), ("q", FvArgF32),
                ("flag", ctypes.c_void_p), ("flag_value", ctypes.c_int8)]


class FvChains(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int64), ("n_maturities", ctypes.c_int64),
                ("n_quotes", ctypes.c_int64),
                ("chain_mat_off", ctypes.c_void_p), ("mat_quote_off", ctypes.c_void_p),
                ("F", ctypes.c_void_p), ("r", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("price", ctypes.c_void_p), ("K", ctypes.c_void_p), ("flag", ctypes.c_void_p)]


class FvSviProblem(ctypes.Structure):
    _fields_ = [("chains", FvChains), ("iv_target", ctypes.c_void_p), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


EXPORTS = ["fv_price", "fv_implied_vol", "fv_implied_vol_f32", "fv_greeks", "fv_implied_vol_backward", "fv_price_backward",
           "fv_implied_vol_chains", "fv_normalised_black", "fv_lbr_trace", "fv_halley_trace", "fv_set_halley_steps", "fv_get_halley_steps",
           "fv_set_launch", "fv_get_launch",
           "fv_autotune", "fv_launch_shape", "fv_tuning_reset", "fv_tuning_save", "fv_tuning_load",
           "fv_svi_workspace_size", "fv_svi_adam_step", "fv_svi_adam_step_noalloc", "fv_svi_vols", "fv_last_error", "fv_version"]

_lib = None


class FastvolError(RuntimeError):
    pass


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FastvolError(
            "libfastvol.so is not built (%s); run paper_2604_27210_amd/build.py "
            "or __graft_entry__.build()" % LIB_PATH)
    import torch  # noqa: F401  -- binds the library to torch's HIP runtime
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, V = ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.fv_price.argtypes = [I, P(FvQuotes), FvArg, V, V]
    lib.fv_implied_vol.argtypes = [I, I, P(FvQuotes), V, V, V, V]
    lib.fv_implied_vol_f32.argtypes = [I, P(FvQuotesF32), V, V, V]
    lib.fv_greeks.argtypes = [I, P(FvQuotes), FvArg, V, V, V, V, V, V]
    lib.fv_implied_vol_backward.argtypes = [I, P(FvQuotes), V, V, V, V, V, V, V, V, V]
    lib.fv_price_backward.argtypes = [I, P(FvQuotes), FvArg, V, V, V, V, V, V, V, V]
    lib.fv_implied_vol_chains.argtypes = [I, P(FvChains), V, V, V]
    lib.fv_normalised_black.argtypes = [I64, V, V, V, V, V]
    lib.fv_lbr_trace.argtypes = [I, P(FvQuotes), V, V]
    lib.fv_halley_trace.argtypes = [I, P(FvQuotes), V, V]
    lib.fv_set_halley_steps.argtypes = [I]
    lib.fv_get_halley_steps.argtypes = []
    lib.fv_svi_workspace_size.argtypes = [P(FvSviProblem)]
    lib.fv_svi_workspace_size.restype = I64
    lib.fv_svi_adam_step.argtypes = [P(FvSviProblem), V, V, V, V, V, V, I64, V, I64, V]
    lib.fv_svi_adam_step_noalloc.argtypes = [P(FvSviProblem), V, V, V, V, V, V, I64, V]
    lib.fv_svi_vols.argtypes = [P(FvSviProblem), V, V, V]
    lib.fv_set_launch.argtypes = [I, I, I]
    lib.fv_get_launch.argtypes = [I, P(I), P(I)]
    lib.fv_autotune.argtypes = [I, I, I64, V]
    lib.fv_launch_shape.argtypes = [I, I, I64, P(I), P(I)]
    lib.fv_tuning_reset.argtypes = []
    lib.fv_tuning_save.argtypes = [ctypes.c_char_p]
    lib.fv_tuning_load.argtypes = [ctypes.c_char_p]
    lib.fv_last_error.argtypes = []
    lib.fv_version.argtypes = []
    for name in EXPORTS:
        getattr(lib, name).restype = I
    lib.fv_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != FV_OK:
        msg = load().fv_last_error().decode(errors="replace")
        raise FastvolError("%s failed (%d): %s" % (what, rc, msg))
