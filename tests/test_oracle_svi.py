"""Pins of the numpy SVI-calibration reference (oracle/svi.py)."""
import numpy as np

from oracle import svi
from paper_2604_27210_amd import workloads as W


def _raw(th):
    out = th.copy()
    out[:, 1] = np.log(np.expm1(th[:, 1]))
    out[:, 2] = np.arctanh(th[:, 2])
    out[:, 4] = np.log(np.expm1(th[:, 4]))
    return out


def _problem(n_chains=6, seed=5):
    c = W.svi_calibration(n_chains, seed)
    ch = c.chains
    mat = ch.mat_of_quote()
    return c, ch.k, mat, ch.T


def test_parametrisation_round_trip_and_vertex():
    c, k, mat, T = _problem()
    a, b, rho, m, s = svi.natural(_raw(c.theta_true))
    np.testing.assert_allclose(np.stack([a, b, rho, m, s], 1), c.theta_true, rtol=1e-13, atol=1e-15)
    # at k = m the total variance is a + b s
    raw = _raw(c.theta_true)
    w = svi.svi_total_variance(raw, m[mat], mat)
    np.testing.assert_allclose(w, a[mat] + b[mat] * s[mat], rtol=1e-14)


def test_gradient_matches_central_differences():
    c, k, mat, T = _problem()
    rng = np.random.default_rng(0)
    target = svi.svi_vols(_raw(c.theta_true), k, mat, T) * (1 + c.eps)
    raw = _raw(c.theta0)
    L, G = svi.loss_and_grad(raw, k, mat, T, target)
    for _ in range(25):
        i, j = rng.integers(raw.shape[0]), rng.integers(5)
        h = 1e-6
        rp, rm = raw.copy(), raw.copy()
        rp[i, j] += h
        rm[i, j] -= h
        fd = (svi.loss_and_grad(rp, k, mat, T, target)[0] - svi.loss_and_grad(rm, k, mat, T, target)[0]) / (2 * h)
        assert abs(fd - G[i, j]) <= 2e-5 * abs(G[i, j]) + 1e-13, (i, j, fd, G[i, j])


def test_adam_first_step_moves_by_lr_and_loss_falls():
    c, k, mat, T = _problem()
    target = svi.svi_vols(_raw(c.theta_true), k, mat, T) * (1 + c.eps)
    raw0 = _raw(c.theta0)
    th1, _ = svi.adam_replay(raw0, k, mat, T, target, 1, lr=1e-2)
    _, G = svi.loss_and_grad(raw0, k, mat, T, target)
    # the bias corrections make m^ = g and v^ = g^2 after one step, so the
    # first move is lr g / (|g| + eps): lr in magnitude wherever |g| >> eps
    np.testing.assert_allclose(raw0 - th1, 1e-2 * G / (np.abs(G) + 1e-8), rtol=1e-12, atol=1e-18)
    big = np.abs(G) > 1e-4
    np.testing.assert_allclose(np.abs(raw0 - th1)[big], 1e-2, rtol=1e-4)
    th, losses = svi.adam_replay(raw0, k, mat, T, target, 200)
    assert losses[-1] < 0.05 * losses[0]
