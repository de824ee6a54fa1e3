"""SVI calibration through the differentiable implied volatility, one or
more Adam steps per replay of a captured hipGraph (torch.cuda.CUDAGraph is
hipGraph on ROCm).  All arithmetic is in ``fv_svi_adam_step`` (four kernel launches,
no allocation, no host synchronisation); this module only owns the device
buffers (state and workspace), the capture and the replays.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _native as N
from . import api


def raw_from_natural(theta_nat: np.ndarray) -> np.ndarray:
    """(a, b, rho, m, s) -> raw (a, b~, rho~, m, s~) with b = softplus(b~),
    rho = tanh(rho~), s = softplus(s~)."""
    t = np.asarray(theta_nat, dtype=np.float64)
    out = t.copy()
    out[:, 1] = np.log(np.expm1(t[:, 1]))
    out[:, 2] = np.arctanh(t[:, 2])
    out[:, 4] = np.log(np.expm1(t[:, 4]))
    return out


class SviCalibrator:
    """Device state of one calibration problem (ragged Black-76 chains)."""

    def __init__(self, chain_mat_off, mat_quote_off, F, r, T, K, flag, iv_target,
                 theta0_raw, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, max_steps=1024):
        dev = F.device
        self.keep = [chain_mat_off, mat_quote_off, F, r, T, K, flag, iv_target]
        for t, nm, dt in ((chain_mat_off, "chain_mat_off", torch.int64),
                          (mat_quote_off, "mat_quote_off", torch.int64), (F, "F", torch.float64),
                          (r, "r", torch.float64), (T, "T", torch.float64), (K, "K", torch.float64),
                          (flag, "flag", torch.int8), (iv_target, "iv_target", torch.float64)):
            api._dev_tensor(t, nm, dt)
        self.n_mat = T.numel()
        self.n = K.numel()
        ch = N.FvChains(F.numel(), self.n_mat, self.n, api._ptr(chain_mat_off),
                        api._ptr(mat_quote_off), api._ptr(F), api._ptr(r), api._ptr(T), None,
                        api._ptr(K), api._ptr(flag))
        self.problem = N.FvSviProblem(ch, api._ptr(iv_target), lr, beta1, beta2, eps)
        th = torch.as_tensor(np.ascontiguousarray(theta0_raw, dtype=np.float64).reshape(-1))
        self.theta = th.to(dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step_count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.grad = torch.empty_like(self.theta)
        nws = N.load().fv_svi_workspace_size(ctypes.byref(self.problem))
        if nws < 0:
            N.check(int(nws), "fv_svi_workspace_size")
        self.workspace = torch.empty(int(nws), dtype=torch.float64, device=dev)
        self.loss = torch.full((max_steps,), float("nan"), dtype=torch.float64, device=dev)
        self.graph = None
        self.steps_per_replay = 0

    def step(self):
        N.check(N.load().fv_svi_adam_step(
            ctypes.byref(self.problem), api._ptr(self.theta), api._ptr(self.m), api._ptr(self.v),
            api._ptr(self.step_count), api._ptr(self.grad), api._ptr(self.workspace),
            self.workspace.numel(), api._ptr(self.loss), self.loss.numel(), ctypes.c_void_p(api._stream_ptr())),
            "fv_svi_adam_step")

    def capture(self, steps_per_replay: int = 1):
        """Capture `steps_per_replay` consecutive steps into one graph (the
        state buffers are updated in place by every replay).  The capture
        itself runs no step.  More than one step per replay spreads the
        runtime's fixed cost of a graph launch over several steps."""
        k = int(steps_per_replay)
        if k < 1:
            raise ValueError("steps_per_replay must be >= 1, got %r" % (steps_per_replay,))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(k):
                self.step()
        self.graph = g
        self.steps_per_replay = k
        return g

    def replay(self):
        self.graph.replay()

    def vols(self, theta=None) -> torch.Tensor:
        th = self.theta if theta is None else theta
        out = torch.empty(self.n, dtype=torch.float64, device=self.theta.device)
        N.check(N.load().fv_svi_vols(ctypes.byref(self.problem), api._ptr(th), api._ptr(out),
                                     ctypes.c_void_p(api._stream_ptr())), "fv_svi_vols")
        return out

    def losses(self) -> np.ndarray:
        k = int(self.step_count.item())
        return self.loss[:min(k, self.loss.numel())].cpu().numpy()


def calibrate_svi(cal: SviCalibrator, steps: int = 200, graph: bool = True,
                  steps_per_replay: int = 1) -> dict:
    """Run `steps` Adam steps (graph replays of `steps_per_replay` steps
    each, or eager launches) and time them."""
    if graph:
        if steps % steps_per_replay:
            raise ValueError("steps (%d) must be a multiple of steps_per_replay (%d)"
                             % (steps, steps_per_replay))
        if cal.graph is None or cal.steps_per_replay != steps_per_replay:
            cal.capture(steps_per_replay)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if graph:
        for _ in range(steps // steps_per_replay):
            cal.replay()
    else:
        for _ in range(steps):
            cal.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"steps": steps, "seconds": dt, "steps_per_s": steps / dt, "graph": graph,
            "steps_per_replay": steps_per_replay if graph else 0}
