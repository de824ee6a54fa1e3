"""Seeded synthetic workloads (the input recipes only).

Each generator draws the *market inputs* of a workload -- spot or forward,
strike, maturity, rates, the true volatility, the option flag and, for the
ragged workloads, the chain / maturity offsets -- with numpy's PCG64
``default_rng(seed)`` in a fixed order.  It computes no price and solves
nothing: the caller turns ``sigma_true`` into input prices with whichever
pricer it is testing or timing, so the same input bits can feed both the GPU
library and an independent reference.

Workload shapes follow the paper's use cases (section 1: whole option chains
across strikes and maturities; section 4: batched inversion at large N).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# injected-quote kinds of the wide Black-Scholes-Merton workload
KIND_CLEAN, KIND_AT, KIND_BELOW, KIND_ABOVE = 0, 1, 2, 3


@dataclass
class Flat:
    """Struct-of-arrays quote batch (all float64 except ``flag``/``kind``)."""
    model: str                 # "black76" | "bs" | "bsm"
    fs: np.ndarray             # forward (black76) or spot
    K: np.ndarray
    T: np.ndarray
    r: np.ndarray
    q: np.ndarray
    sigma_true: np.ndarray
    flag: np.ndarray           # int8, +1 call / -1 put
    kind: np.ndarray = None    # uint8 KIND_* (None: all clean)
    pert: np.ndarray = None    # uniform draw used by an injected quote
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.K.shape[0])

    def take(self, idx) -> "Flat":
        sub = lambda a: None if a is None else a[idx]
        return Flat(self.model, self.fs[idx], self.K[idx], self.T[idx], self.r[idx],
                    self.q[idx], self.sigma_true[idx], self.flag[idx], sub(self.kind),
                    sub(self.pert), dict(self.extra))


@dataclass
class Chains:
    """Ragged Black-76 option chains in CSR form.

    chain_mat_off[c]..chain_mat_off[c+1] are the maturities of chain c;
    mat_quote_off[m]..mat_quote_off[m+1] are the quotes of maturity m.
    F, r are per chain; T is per maturity; K, flag, sigma_true per quote.
    """
    chain_mat_off: np.ndarray  # int64 [n_chains+1]
    mat_quote_off: np.ndarray  # int64 [n_mat+1]
    F: np.ndarray              # [n_chains]
    r: np.ndarray              # [n_chains]
    T: np.ndarray              # [n_mat]
    K: np.ndarray              # [n_quotes]
    flag: np.ndarray           # int8 [n_quotes]
    sigma_true: np.ndarray     # [n_quotes]
    k: np.ndarray              # log-moneyness ln(K/F) per quote [n_quotes]

    @property
    def n_chains(self) -> int:
        return int(self.F.shape[0])

    @property
    def n_mat(self) -> int:
        return int(self.T.shape[0])

    @property
    def n(self) -> int:
        return int(self.K.shape[0])

    def mat_of_quote(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_mat), np.diff(self.mat_quote_off))

    def chain_of_mat(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_chains), np.diff(self.chain_mat_off))

    def flatten(self) -> Flat:
        """Expand per-chain / per-maturity fields to one row per quote."""
        m = self.mat_of_quote()
        c = self.chain_of_mat()[m]
        return Flat("black76", self.F[c], self.K.copy(), self.T[m], self.r[c],
                    np.zeros(self.n), self.sigma_true.copy(), self.flag.copy())


def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def bs_small(n: int = 4096, seed: int = 1) -> Flat:
    """Black-Scholes, small batch: S=100; K = S e^u, u~U[-0.5,0.5];
    T~U[0.02,2]; r~U[0,0.05]; q=0; sigma~U[0.05,1]; call/put 50/50."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-0.5, 0.5, n)
    T = rng.uniform(0.02, 2.0, n)
    r = rng.uniform(0.0, 0.05, n)
    sig = rng.uniform(0.05, 1.0, n)
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    S = np.full(n, 100.0)
    return Flat("bs", S, 100.0 * np.exp(u), T, r, np.zeros(n), sig, flag)


def bsm_wide(n: int = 10_000_000, seed: int = 2, zmax: float = 6.0,
             inject: float = 0.01) -> Flat:
    """Black-Scholes-Merton, wide wings: S=100; ln(F/K) = z sigma sqrt(T) with
    z~U[-zmax,zmax]; sigma~logU[0.01,3]; T~logU[1/365,5]; r~U[-0.01,0.08];
    q~U[0,0.05]; call/put 50/50.  A fraction ``inject`` of the quotes is
    marked for a degenerate price, split 40/30/30 between at-intrinsic,
    below-intrinsic and above-the-upper-bound (``kind``), each with a uniform
    draw ``pert`` in [1e-6, 1e-2] (below) or [1e-6, 0.1] (above)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-zmax, zmax, n)
    sig = _loguniform(rng, 0.01, 3.0, n)
    T = _loguniform(rng, 1.0 / 365.0, 5.0, n)
    r = rng.uniform(-0.01, 0.08, n)
    q = rng.uniform(0.0, 0.05, n)
    flag = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
    S = np.full(n, 100.0)
    F = S * np.exp((r - q) * T)
    K = F * np.exp(-z * sig * np.sqrt(T))
    kind = np.zeros(n, dtype=np.uint8)
    pert = np.zeros(n)
    n_inj = int(round(inject * n))
    if n_inj:
        idx = rng.choice(n, size=n_inj, replace=False)
        n_at = int(round(0.4 * n_inj))
        n_below = int(round(0.3 * n_inj))
        kind[idx[:n_at]] = KIND_AT
        kind[idx[n_at:n_at + n_below]] = KIND_BELOW
        kind[idx[n_at + n_below:]] = KIND_ABOVE
        pb = rng.uniform(1e-6, 1e-2, n_below)
        pa = rng.uniform(1e-6, 0.1, n_inj - n_at - n_below)
        pert[idx[n_at:n_at + n_below]] = pb
        pert[idx[n_at + n_below:]] = pa
    out = Flat("bsm", S, K, T, r, q, sig, flag, kind, pert)
    out.extra["z"] = z
    return out


def bsm_diff(n: int = 1_000_000, seed: int = 4) -> Flat:
    """Differentiation workload: as ``bsm_wide`` with |z| <= 3 and no
    injections, plus loss weights w~N(0,1) in ``extra['w']``."""
    out = bsm_wide(n, seed=seed, zmax=3.0, inject=0.0)
    rng = np.random.default_rng(seed + 1000)
    out.extra["w"] = rng.standard_normal(n)
    return out


def b76_chains(n_chains: int = 2000, seed: int = 3) -> Chains:
    """Ragged Black-76 chains: per chain 1..30 maturities (uniform integer),
    T sorted draws from logU[1/365,5], F~U[10,5000], r~U[0,0.05]; per maturity
    clip(round(logN(ln 200, 0.8)), 20, 2000) strikes on a uniform grid in
    k = ln(K/F) over [-1.2 sqrt(T), 1.2 sqrt(T)]; smile
    sigma = 0.2 + 0.1 k^2 - 0.05 k; out-of-the-money flags (put if K < F)."""
    rng = np.random.default_rng(seed)
    n_mat_per_chain = rng.integers(1, 31, n_chains)
    F = rng.uniform(10.0, 5000.0, n_chains)
    r = rng.uniform(0.0, 0.05, n_chains)
    n_mat = int(n_mat_per_chain.sum())
    chain_mat_off = np.zeros(n_chains + 1, dtype=np.int64)
    chain_mat_off[1:] = np.cumsum(n_mat_per_chain)
    T = _loguniform(rng, 1.0 / 365.0, 5.0, n_mat)
    for c in range(n_chains):
        a, b = chain_mat_off[c], chain_mat_off[c + 1]
        T[a:b] = np.sort(T[a:b])
    n_k = np.clip(np.round(rng.lognormal(np.log(200.0), 0.8, n_mat)), 20, 2000).astype(np.int64)
    mat_quote_off = np.zeros(n_mat + 1, dtype=np.int64)
    mat_quote_off[1:] = np.cumsum(n_k)
    n = int(mat_quote_off[-1])
    mat = np.repeat(np.arange(n_mat), n_k)
    chain = np.repeat(np.arange(n_chains), n_mat_per_chain)[mat]
    # position j of each quote within its maturity, on a uniform k grid
    j = np.arange(n) - mat_quote_off[mat]
    width = 1.2 * np.sqrt(T[mat])
    k = -width + 2.0 * width * j / np.maximum(n_k[mat] - 1, 1)
    K = F[chain] * np.exp(k)
    sig = 0.2 + 0.1 * k * k - 0.05 * k
    flag = np.where(K < F[chain], -1, 1).astype(np.int8)
    return Chains(chain_mat_off, mat_quote_off, F, r, T, K, flag, sig, k)


@dataclass
class SviCalibration:
    """Calibration workload: ragged Black-76 chains plus per-maturity SVI
    parameters in natural units (a, b, rho, m, s) -- the generating set
    ``theta_true`` and a perturbed starting point ``theta0`` -- and the
    relative noise ``eps`` that perturbs each target volatility."""
    chains: Chains
    theta_true: np.ndarray   # [n_mat, 5]
    theta0: np.ndarray       # [n_mat, 5]
    eps: np.ndarray          # [n_quotes]


SVI_RANGES = np.array([[0.005, 0.03], [0.05, 0.3], [-0.7, 0.0], [-0.1, 0.1], [0.05, 0.3]])


def svi_calibration(n_chains: int = 500, seed: int = 5) -> SviCalibration:
    """Chains as ``b76_chains``; per maturity a~U[0.005,0.03], b~U[0.05,0.3],
    rho~U[-0.7,0], m~U[-0.1,0.1], s~U[0.05,0.3]; start = truth + N(0, (20% of
    each range)^2), clipped into the range; eps~N(0, 0.01^2) per quote."""
    ch = b76_chains(n_chains, seed=seed)
    rng = np.random.default_rng(seed + 100)
    lo, hi = SVI_RANGES[:, 0], SVI_RANGES[:, 1]
    th = lo + (hi - lo) * rng.random((ch.n_mat, 5))
    th0 = np.clip(th + rng.standard_normal((ch.n_mat, 5)) * 0.2 * (hi - lo), lo, hi)
    eps = rng.normal(0.0, 0.01, ch.n)
    return SviCalibration(ch, th, th0, eps)
