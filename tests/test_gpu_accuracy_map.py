"""Dense (x, s) plane: the normalised Black evaluator and both solvers
against the oracle everywhere the price is solvable (see accuracy_map.py)."""
import numpy as np
import pytest

import accuracy_map as AM
from _helpers import boundary_ambiguous

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2604_27210_amd as fv
    fv._native.load()
    return fv


def test_plane_within_bounds(fv):
    nx = ns = 64
    xs, ss, res, ok = AM.measure(fv, torch, nx, ns)
    _, _, x, s = AM.plane(nx, ns)
    assert ok.sum() > 0.6 * ok.size
    # every solvable cell is compared against a finite tolerance, including
    # the cells whose price lies below the normal binary64 range
    assert res["inf_tol"] == 0
    assert res["subnormal_price_cells"] > 0
    # b: a few ulps of the exact b at the given (x, s) everywhere, the deep
    # wing included (the exponent -(h^2 + t^2)/2 is formed to twice the
    # working precision, so the rounding of h = x/s is not amplified by h^2);
    # below the normal range a few units of the smallest subnormal on top
    bo = AM.oracle.normalised_black(x, s, 1)
    bound = 16.0 + np.where(bo < 2.2250738585072014e-308, 4.0 * 2.0**-1074 / np.maximum(bo, 2.0**-1074), 0.0) / AM.U
    eb = res["b"]
    m = np.isfinite(eb)
    assert m.sum() > 0.6 * m.size
    assert np.all(eb[m] <= bound[m]), (np.max(eb[m] / bound[m]), x[m][np.argmax(eb[m] / bound[m])])
    for solver in ("lbr", "halley"):
        r = res[solver + "_ratio"]
        assert np.nanmax(r) <= 1.0, (solver, np.nanmax(r))
        # solved cells are compared; no solvable cell is left unsolved except
        # by a boundary-ambiguous status (checked below)
        assert np.all(np.isfinite(r[ok]) | np.isin(np.where(ok)[0], res[solver + "_status_mismatch"]))
        mis = res[solver + "_status_mismatch"]
        if len(mis):
            K = np.exp(-x[mis])
            one = np.ones(len(mis))
            P = AM.oracle.price("black76", one, K, one, 0 * one, 0.0, s[mis],
                                np.ones(len(mis), dtype=np.int8))
            amb = boundary_ambiguous("black76", P, one, K, one, 0 * one, 0.0,
                                     np.ones(len(mis), dtype=np.int8))
            assert np.all(amb), (solver, x[mis][~amb][:5], s[mis][~amb][:5])
