"""Gradient of a sparse-probe velocity misfit with respect to the inflow profile.

The forward run is the HIP solver; the backward run is the hand-written
discrete adjoint (lbm_adjoint_step) driven here with checkpointing:

* forward: set u_in(z) = s_z (cos theta, sin theta, 0) on one inflow face,
  start from the fixed initial state, store the canonical state every K
  steps (checkpoints), and accumulate u at the registered probe cells after
  every step; output u_bar = (1/T) sum_{t=1..T} u(x_p, t);
* backward: for each segment in reverse, recompute the K + 1 states of the
  segment from its checkpoint with the out-of-place push step, then run the
  adjoint steps t = segment end .. segment start + 1 (and t = 0 for the first
  segment) with the probe source dL/du(x_p, t) = g_ubar / T for t >= 1;
  the per-height inflow gradient accumulates in a compensated sum, and the
  chain rule through u_in(z) gives d/ds_z and d/dtheta.

The initial state is held fixed (not differentiated).  Python only marshals
arguments and orders the calls; every step and adjoint step runs on the GPU.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding


class InflowProblem:
    """A solver context plus everything the forward/backward pair needs."""

    def __init__(self, lat: binding.LBM, probes, steps: int, every: int, u0, face: int = 0):
        if steps % every != 0:
            raise ValueError("steps must be a multiple of the checkpoint interval")
        self.lat = lat
        self.probes = np.ascontiguousarray(probes, np.int32).reshape(-1, 3)
        lat.set_probes(self.probes)
        self.T = int(steps)
        self.K = int(every)
        self.u0 = np.asarray(u0, np.float64)
        self.face = int(face)
        self.nz = lat.nz
        self.device = lat.device
        self.rdt = lat.real_dtype
        self.forward_calls = 0
        self.backward_calls = 0

    def profile(self, speeds: np.ndarray, theta: float) -> np.ndarray:
        s = np.asarray(speeds, np.float64)
        return np.stack([s * math.cos(theta), s * math.sin(theta), np.zeros_like(s)], axis=1)

    def run_forward(self, speeds, theta, keep_checkpoints=True):
        lat = self.lat
        lat.set_inflow(self.face, self.profile(speeds, theta))
        lat.reset(self.u0)
        acc = torch.zeros(2, self.probes.shape[0], 3, dtype=self.rdt, device=self.device)   # sum, compensation
        ckpts = []
        for _ in range(self.T // self.K):
            if keep_checkpoints:
                ckpts.append(lat.get_state()[0])          # a fresh tensor per checkpoint
            lat.step_probed(self.K, acc)
        self.forward_calls += 1
        return (acc[0].double() + acc[1].double()) / self.T, ckpts

    def run_backward(self, ckpts, g_ubar: torch.Tensor, speeds, theta):
        """Returns (d/d speeds [nz], d/d theta) as float64 numpy values."""
        lat = self.lat
        T, K = self.T, self.K
        src = (g_ubar.to(self.device, self.rdt) / T).contiguous()
        lam_next = torch.zeros(19, lat.nz, lat.ny, lat.nx, dtype=self.rdt, device=self.device)
        lam = torch.empty_like(lam_next)
        g = torch.zeros(2, 6, lat.nz, 3, dtype=self.rdt, device=self.device)
        work = [lat.new_state() for _ in range(K)]
        for seg in range(T // K - 1, -1, -1):
            t0 = seg * K
            snaps = [ckpts[seg]] + work          # the checkpoint is only read
            for k in range(K):
                lat.push_step(snaps[k], snaps[k + 1])
            last = t0 + K
            first = t0 if seg == 0 else t0 + 1
            for t in range(last, first - 1, -1):
                lat.adjoint_step(snaps[t - t0], lam_next, lam, src if t >= 1 else None, g)
                lam_next, lam = lam, lam_next
        self.backward_calls += 1
        gz = (g[0, self.face].double() + g[1, self.face].double()).cpu().numpy()   # [nz, 3]
        c, s = math.cos(theta), math.sin(theta)
        sp = np.asarray(speeds, np.float64)
        d_speeds = gz[:, 0] * c + gz[:, 1] * s
        d_theta = float((gz[:, 0] * (-sp * s) + gz[:, 1] * (sp * c)).sum())
        return d_speeds, d_theta


class LBMInflow(torch.autograd.Function):
    """u_bar [np, 3] = time-averaged probe velocities for inflow speeds [nz]
    and angle theta (radians) on the problem's inflow face."""

    @staticmethod
    def forward(ctx, speeds: torch.Tensor, theta: torch.Tensor, problem: InflowProblem):
        sp = speeds.detach().double().cpu().numpy()
        th = float(theta.detach().double().cpu())
        ubar, ckpts = problem.run_forward(sp, th)
        ctx.problem = problem
        ctx.ckpts = ckpts
        ctx.sp, ctx.th = sp, th
        ctx.sdtype, ctx.sdev = speeds.dtype, speeds.device
        return ubar.to(speeds.device)

    @staticmethod
    def backward(ctx, g_ubar: torch.Tensor):
        d_sp, d_th = ctx.problem.run_backward(ctx.ckpts, g_ubar, ctx.sp, ctx.th)
        ctx.ckpts = None
        gs = torch.from_numpy(d_sp).to(ctx.sdev, ctx.sdtype)
        gt = torch.tensor(d_th, dtype=ctx.sdtype, device=ctx.sdev)
        return gs, gt, None


def probe_misfit(problem: InflowProblem, speeds: torch.Tensor, theta: torch.Tensor, target: torch.Tensor):
    """L = sum_p |u_bar_p - target_p|^2 through the adjoint-backed Function."""
    ubar = LBMInflow.apply(speeds, theta, problem)
    return ((ubar - target.to(ubar.device, ubar.dtype)) ** 2).sum()
