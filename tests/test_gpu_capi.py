"""The C ABI from plain C: `fv_capi_demo` (built by the package build with
gcc, linked against libfastvol.so and the HIP runtime, no Python in the
process) prices a seeded batch, inverts it with both solvers, checks the
round trip against the inversion's conditioning and times the calls.  Run as
a child process; its JSON line carries the checks and the timings."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
DEMO = os.path.join(HERE, "..", "paper_2604_27210_amd", "_build", "fv_capi_demo")


@pytest.fixture(scope="module")
def demo():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(DEMO), "fv_capi_demo is not built (run __graft_entry__.build())"
    return DEMO


@pytest.mark.parametrize("n,reps", [(1, 20), (4096, 200), (1_000_003, 20), (10_000_000, 10)])
def test_c_caller_round_trip(demo, n, reps):
    res = subprocess.run([demo, str(n), str(reps)], capture_output=True, text=True, timeout=180)
    print(res.stdout.strip())
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["ok"] and out["n"] == n
    for solver in ("lbr", "halley"):
        assert out[solver]["bad"] == 0
        assert out[solver]["at_bound"] <= max(1, n // 50)
        assert out[solver]["worst_err_over_tol"] <= 1.0
