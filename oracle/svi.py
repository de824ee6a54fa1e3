"""TEST INFRASTRUCTURE ONLY -- plain numpy reference of the SVI calibration.

The calibration minimises L(theta) = (1/N) sum_i (IV(P(sigma_i(theta))) -
v_i)^2 over per-maturity SVI parameters, with sigma_i = sqrt(w(k_i)/T_i) and
w(k) = a + b (rho (k - m) + sqrt((k - m)^2 + s^2)) (raw parameters
(a, b~, rho~, m, s~), b = softplus(b~), rho = tanh(rho~), s = softplus(s~)).
Since IV(P(sigma)) = sigma exactly (the implied volatility is the root of
the pricing equation, paper section 1), the loss is by definition
(1/N) sum (sigma_i(theta) - v_i)^2 and its gradient is the plain chain rule
written out below.  ``adam_replay`` repeats the optimiser's recurrence
(Kingma & Ba, Adam, 2015) step by step.  Nothing here is shared with the GPU
library.
"""
from __future__ import annotations

import numpy as np


def natural(raw):
    raw = np.asarray(raw, dtype=np.float64)
    a = raw[:, 0]
    b = np.log1p(np.exp(raw[:, 1]))
    rho = np.tanh(raw[:, 2])
    m = raw[:, 3]
    s = np.log1p(np.exp(raw[:, 4]))
    return a, b, rho, m, s


def svi_total_variance(raw, k, mat):
    """w per quote; k = ln(K/F) per quote, mat = maturity index per quote."""
    a, b, rho, m, s = natural(raw)
    dk = k - m[mat]
    return a[mat] + b[mat] * (rho[mat] * dk + np.sqrt(dk * dk + s[mat] ** 2))


def svi_vols(raw, k, mat, T):
    w = svi_total_variance(raw, k, mat)
    with np.errstate(invalid="ignore"):
        return np.sqrt(w / T[mat])


def loss_and_grad(raw, k, mat, T, target):
    """L and dL/draw [n_mat, 5], over quotes with w > 1e-10 and finite
    target, normalised by the total number of quotes."""
    raw = np.asarray(raw, dtype=np.float64)
    n_mat = raw.shape[0]
    a, b, rho, m, s = natural(raw)
    dk = k - m[mat]
    rt = np.sqrt(dk * dk + s[mat] ** 2)
    w = a[mat] + b[mat] * (rho[mat] * dk + rt)
    ok = (w > 1e-10) & np.isfinite(target)
    sig = np.sqrt(np.where(ok, w, 1.0) / T[mat])
    e = np.where(ok, sig - target, 0.0)
    N = k.shape[0]
    L = np.sum(e * e) / N
    g_w = np.where(ok, 2.0 * e / N / (2.0 * sig * T[mat]), 0.0)
    sg = lambda z: 1.0 / (1.0 + np.exp(-z))
    dw = np.stack([np.ones_like(dk),
                   (rho[mat] * dk + rt) * sg(raw[mat, 1]),
                   b[mat] * dk * (1.0 - rho[mat] ** 2),
                   b[mat] * (-rho[mat] - dk / rt),
                   b[mat] * (s[mat] / rt) * sg(raw[mat, 4])], 1)
    G = np.zeros((n_mat, 5))
    for j in range(5):
        G[:, j] = np.bincount(mat, weights=g_w * dw[:, j], minlength=n_mat)
    return L, G


def adam_replay(raw0, k, mat, T, target, steps, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """theta after `steps` Adam steps and the loss before each step."""
    th = np.array(raw0, dtype=np.float64)
    mo = np.zeros_like(th)
    vo = np.zeros_like(th)
    losses = []
    for t in range(1, steps + 1):
        L, G = loss_and_grad(th, k, mat, T, target)
        losses.append(L)
        mo = b1 * mo + (1 - b1) * G
        vo = b2 * vo + (1 - b2) * G * G
        mh = mo / (1 - b1 ** t)
        vh = vo / (1 - b2 ** t)
        th = th - lr * mh / (np.sqrt(vh) + eps)
    return th, np.array(losses)
