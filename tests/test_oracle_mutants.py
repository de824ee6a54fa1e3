"""The oracle's pins catch plausible mistakes (CPU only): the binary128 C
oracle and the numpy calibration reference.

Each mutant is fv_oracle.c with one deliberate slip -- a dropped term, a
wrong sign, a swapped operand or index, a put branch that lost its flag --
compiled into a library of its own; the pin suite (tests/test_oracle_pins.py)
then runs against it in a child process (FV_ORACLE_LIB selects the build)
and must fail.  The unmutated oracle passes the same suite in the main run.
The mistakes are planted in the oracle's source text, on the CPU; nothing
here touches the GPU library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINS = os.path.join(HERE, "test_oracle_pins.py")

# (what goes wrong, the oracle's text, the mistaken text)
MUTANTS = [
    ("Black-76 price not discounted",
     "return D * th * (a->fs * q_Phi(th * d1) - a->K * q_Phi(th * d2));",
     "return th * (a->fs * q_Phi(th * d1) - a->K * q_Phi(th * d2));"),
    ("Black-76 d2 = d1 + s",
     "qr d1 = (logq(a->fs / a->K) + 0.5Q * sigma * sigma * a->T) / sd;\n        qr d2 = d1 - sd;",
     "qr d1 = (logq(a->fs / a->K) + 0.5Q * sigma * sigma * a->T) / sd;\n        qr d2 = d1 + sd;"),
    ("BSM price: carry r + q",
     "(logq(a->fs / a->K) + (a->r - qy + 0.5Q * sigma * sigma) * a->T) / sd;",
     "(logq(a->fs / a->K) + (a->r + qy + 0.5Q * sigma * sigma) * a->T) / sd;"),
    ("forward: carry r + q",
     "qr carry = (a->model == ORC_BSM) ? (a->r - a->q) : a->r;",
     "qr carry = (a->model == ORC_BSM) ? (a->r + a->q) : a->r;"),
    ("BSM put: Phi(d2) without the flag",
     "- a->K * D * q_Phi(th * d2));",
     "- a->K * D * q_Phi(d2));"),
    ("BSM vega without sqrt(T)",
     "out[2] = S * Dq * q_phi(d1) * sqT;",
     "out[2] = S * Dq * q_phi(d1);"),
    ("BSM gamma without sigma",
     "out[1] = Dq * q_phi(d1) / (S * sigma * sqT);",
     "out[1] = Dq * q_phi(d1) / (S * sqT);"),
    ("Black-76 theta: sign of r P",
     "out[3] = a->r * P - D * F * q_phi(d1) * sigma / (2 * sqT);",
     "out[3] = -a->r * P - D * F * q_phi(d1) * sigma / (2 * sqT);"),
    ("Black-76 rho: sign",
     "out[4] = -a->T * P;",
     "out[4] = a->T * P;"),
    ("dP/dK with d1",
     "dP[1] = -th * D * q_Phi(th * d2);",
     "dP[1] = -th * D * q_Phi(th * d1);"),
    ("IV gradient: sign of dsigma/dX",
     "g[1 + j] = (double)(-dP[j] / v);",
     "g[1 + j] = (double)(dP[j] / v);"),
    ("normalised Black: e^{x/2} and e^{-x/2} swapped",
     "b = th * (expq(X / 2) * q_Phi(th * (h + t)) - expq(-X / 2) * q_Phi(th * (h - t)));",
     "b = th * (expq(-X / 2) * q_Phi(th * (h + t)) - expq(X / 2) * q_Phi(th * (h - t)));"),
    ("relative sensitivity: price term without the price",
     "e[0] = (double)((qr)price[i] / v);",
     "e[0] = (double)(1 / v);"),
    ("relative sensitivity: sign of the input terms",
     "e[1 + j] = (double)(-dP[j] * X[j] / v);",
     "e[1 + j] = (double)(dP[j] * X[j] / v);"),
    ("gradient at a given sigma: 1/vega dropped from the input terms",
     "row[1 + j] = (double)(-dP[j] / v);",
     "row[1 + j] = (double)(-dP[j]);"),
    ("status: upper bound of a put is F",
     "double M = theta > 0 ? F : K;",
     "double M = theta > 0 ? F : F;"),
]


def _run_pins(tag, name, old, new, workdir):
    with open(oracle._SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, "mutation site not unique: " + name
    csrc = os.path.join(workdir, tag + ".c")
    with open(csrc, "w") as fh:
        fh.write(src.replace(old, new))
    lib = oracle.build(src=csrc, out=os.path.join(workdir, "lib" + tag + ".so"))
    env = dict(os.environ, FV_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider",
                          "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=900)
    return name, res.returncode, res.stdout[-1500:]


# Slips in the numpy SVI reference (oracle/svi.py), caught by
# tests/test_oracle_svi.py: each runs from a temporary copy of the oracle
# package whose svi.py carries the slip, placed first on the import path.
SVI_MUTANTS = [
    ("softplus derivative of b~ at -b~",
     "(rho[mat] * dk + rt) * sg(raw[mat, 1])", "(rho[mat] * dk + rt) * sg(-raw[mat, 1])"),
    ("tanh derivative dropped from d/drho~",
     "b[mat] * dk * (1.0 - rho[mat] ** 2)", "b[mat] * dk"),
    ("d/dm: sign of the root term",
     "b[mat] * (-rho[mat] - dk / rt)", "b[mat] * (-rho[mat] + dk / rt)"),
    ("total variance: s instead of s^2 under the root",
     "np.sqrt(dk * dk + s[mat] ** 2))\n", "np.sqrt(dk * dk + s[mat]))\n"),
    ("loss halved",
     "L = np.sum(e * e) / N", "L = np.sum(e * e) / (2 * N)"),
    ("Adam without the second bias correction",
     "vh = vo / (1 - b2 ** t)", "vh = vo"),
]
SVI_PINS = os.path.join(HERE, "test_oracle_svi.py")


def _run_svi_pins(tag, name, old, new, workdir):
    import shutil
    d = os.path.join(workdir, tag)
    pkg = os.path.join(d, "oracle")
    os.makedirs(pkg)
    src_dir = os.path.dirname(oracle._SRC)
    shutil.copy(os.path.join(src_dir, "__init__.py"), pkg)
    with open(os.path.join(src_dir, "svi.py")) as fh:
        src = fh.read()
    assert src.count(old) == 1, "mutation site not unique: " + name
    with open(os.path.join(pkg, "svi.py"), "w") as fh:
        fh.write(src.replace(old, new))
    shutil.copy(SVI_PINS, d)
    env = dict(os.environ, PYTHONPATH=ROOT, FV_ORACLE_LIB=oracle._LIB_PATH)
    res = subprocess.run([sys.executable, "-m", "pytest", "test_oracle_svi.py", "-x", "-q",
                          "-p", "no:cacheprovider"], cwd=d, env=env, capture_output=True,
                         text=True, timeout=900)
    return name, res.returncode, res.stdout[-1500:]


def _check(run, mutants, workdir):
    # job 0 is a control: the same harness on an unchanged copy must pass
    jobs = [("c00", "control: unchanged", mutants[0][1], mutants[0][1])]
    jobs += [("m%02d" % k, *m) for k, m in enumerate(mutants, 1)]
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda j: run(*j, workdir), jobs))
    name, rc, out = results[0]
    assert rc == 0, ("the unchanged copy fails its pins", out)
    # pytest exits 1 when a test failed; anything else (0 = all passed,
    # 2+ = the run itself broke) means the pins did not catch the slip
    survivors = [(name, out) for name, rc, out in results[1:] if rc != 1]
    assert not survivors, survivors


def test_every_svi_mutant_fails_a_pin(tmp_path):
    oracle.build(force=False)
    _check(_run_svi_pins, SVI_MUTANTS, str(tmp_path))


def test_every_mutant_fails_a_pin(tmp_path):
    _check(_run_pins, MUTANTS, str(tmp_path))
