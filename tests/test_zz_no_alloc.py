"""The allocation-free calibration step (fv_svi_adam_step_noalloc, workspace
in the library's own per-device array) against fv_svi_adam_step with a
caller workspace, through the C ABI: two problems in a row, the second
smaller, every output bitwise equal over several steps."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import svi
from paper_2604_27210_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_27210_amd import _native as N
    return N.load()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _raw(th):
    out = th.copy()
    out[:, 1] = np.log(np.expm1(th[:, 1]))
    out[:, 2] = np.arctanh(th[:, 2])
    out[:, 4] = np.log(np.expm1(th[:, 4]))
    return out


def _problem(n_chains, seed):
    from paper_2604_27210_amd import _native as N
    c = W.svi_calibration(n_chains, seed=seed)
    ch = c.chains
    mat = ch.mat_of_quote()
    chain = ch.chain_of_mat()[mat]
    sig = svi.svi_vols(_raw(c.theta_true), ch.k, mat, ch.T) * (1.0 + c.eps)
    P = oracle.price("black76", ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0, sig, ch.flag)
    tgt, st = oracle.implied_vol("black76", P, ch.F[chain], ch.K, ch.T[mat], ch.r[chain], 0.0,
                                 ch.flag)
    keep = [dev(ch.chain_mat_off, torch.int64), dev(ch.mat_quote_off, torch.int64), dev(ch.F),
            dev(ch.r), dev(ch.T), dev(ch.K), dev(ch.flag, torch.int8),
            dev(np.where(st == 0, tgt, np.nan))]
    p = lambda t: t.data_ptr()
    chs = N.FvChains(ch.n_chains, ch.n_mat, ch.n, p(keep[0]), p(keep[1]), p(keep[2]), p(keep[3]),
                     p(keep[4]), None, p(keep[5]), p(keep[6]))
    prob = N.FvSviProblem(chs, p(keep[7]), 1e-2, 0.9, 0.999, 1e-8)
    return prob, keep, _raw(c.theta0).reshape(-1), ch.n_mat


def _state(theta0, n_mat, steps):
    t = lambda a: torch.as_tensor(a, dtype=torch.float64).to("cuda").clone()
    return {"theta": t(theta0), "m": t(np.zeros(5 * n_mat)), "v": t(np.zeros(5 * n_mat)),
            "step": torch.zeros(1, dtype=torch.int64, device="cuda"),
            "grad": t(np.full(5 * n_mat, np.nan)), "loss": t(np.full(steps, np.nan))}


def _run(lib, prob, s, steps, workspace):
    from paper_2604_27210_amd import _native as N
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda k: ctypes.c_void_p(s[k].data_ptr())
    for _ in range(steps):
        if workspace is None:
            rc = lib.fv_svi_adam_step_noalloc(ctypes.byref(prob), p("theta"), p("m"), p("v"),
                                              p("step"), p("grad"), p("loss"), steps, stream)
        else:
            rc = lib.fv_svi_adam_step(ctypes.byref(prob), p("theta"), p("m"), p("v"), p("step"),
                                      p("grad"), ctypes.c_void_p(workspace.data_ptr()),
                                      workspace.numel(), p("loss"), steps, stream)
        assert rc == N.FV_OK, lib.fv_last_error()
    torch.cuda.synchronize()


def test_noalloc_step_equals_workspace_step(lib):
    steps = 6
    # two calls in a row on the library's array: a larger problem, then a
    # smaller one whose run sums sit at other offsets of the same array
    for n_chains, seed in ((40, 5), (7, 11)):
        prob, keep, theta0, n_mat = _problem(n_chains, seed)
        nws = lib.fv_svi_workspace_size(ctypes.byref(prob))
        assert nws > 0
        ws = torch.full((nws,), float("nan"), dtype=torch.float64, device="cuda")
        a = _state(theta0, n_mat, steps)
        b = _state(theta0, n_mat, steps)
        _run(lib, prob, a, steps, ws)
        _run(lib, prob, b, steps, None)
        print("noalloc: %d chains, %d maturities, workspace %d doubles" % (n_chains, n_mat, nws))
        for k in a:
            assert torch.equal(a[k], b[k]), k
        assert int(b["step"].item()) == steps
        assert torch.all(torch.isfinite(b["loss"]))


def test_noalloc_rejects_problems_beyond_its_array(lib):
    from paper_2604_27210_amd import _native as N
    prob, keep, theta0, n_mat = _problem(3, 5)
    big = N.FvSviProblem(N.FvChains(prob.chains.n_chains, prob.chains.n_maturities,
                                    (1 << 20) * 64, prob.chains.chain_mat_off,
                                    prob.chains.mat_quote_off, prob.chains.F, prob.chains.r,
                                    prob.chains.T, None, prob.chains.K, prob.chains.flag),
                         prob.iv_target, 1e-2, 0.9, 0.999, 1e-8)
    s = _state(theta0, n_mat, 1)
    p = lambda k: ctypes.c_void_p(s[k].data_ptr())
    rc = lib.fv_svi_adam_step_noalloc(ctypes.byref(big), p("theta"), p("m"), p("v"), p("step"),
                                      p("grad"), p("loss"), 1, None)
    assert rc == N.FV_E_INVALID_ARG
    assert b"at most" in lib.fv_last_error()
    assert int(s["step"].item()) == 0
