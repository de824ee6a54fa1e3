"""Build the gfx950 shared library ``_build/libfastvol.so`` with hipcc.

The library is linked against ``libamdhip64.so.7``; the Python binding loads
it after importing torch, so the HIP runtime already mapped by torch serves
it (same SONAME) and torch's streams and device pointers are valid in it.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libfastvol.so")
SOURCES = [os.path.join(CSRC, "fv_kernels.hip"), os.path.join(CSRC, "fv_calib.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    "-mcode-object-version=5",
    # packed FP32 instructions stay off (they are not needed by this FP64 code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no two-address v_fmac_f64: with it every polynomial step whose addend is
    # a constant costs a v_mov_b64 copy of that constant (hoisted into VGPRs
    # as well); without it the step is one three-operand v_fma_f64 taking the
    # constant from SGPRs, materialised by scalar moves that issue beside the
    # vector pipe (about 20% fewer vector instructions, half the VGPRs)
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-fno-gpu-rdc",
    "-Wall", "-Wno-unused-function",
]


DEMO_SRC = os.path.join(CSRC, "fv_capi_demo.c")
DEMO = os.path.join(OUT_DIR, "fv_capi_demo")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_capi_demo(verbose: bool = False) -> str:
    """The plain-C caller of the library (gcc, linked against the built
    libfastvol.so and the HIP runtime; no Python involved when it runs)."""
    tmp = DEMO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(HERE, "..", "include"), "-I", os.path.join(ROCM, "include"),
           DEMO_SRC, "-o", tmp, "-L", OUT_DIR, "-lfastvol", "-L", os.path.join(ROCM, "lib"),
           "-lamdhip64", "-lm", "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, DEMO)
    return DEMO


def build(verbose: bool = False, extra=None, out: str = None) -> str:
    lib = out or LIB
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + list(extra or []) + ["-I", os.path.join(HERE, "..", "include")] \
        + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "warnings generated" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
    print(build_capi_demo(verbose=True))
