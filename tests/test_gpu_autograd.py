"""Checkpointed discrete adjoint behind torch.autograd.Function (needs an MI355X).

Loss: sum over probes of |time-averaged u - target|^2, parameters: the
per-height inflow speeds of the x- face and the inflow angle.  Checked
against central finite differences (h = 1e-4) of the FP64 GPU forward, and
against the FP64 CPU oracle adjoint over a short trajectory.
"""
import math

import numpy as np
import pytest
import torch

from helpers import oracle_for
from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")
adjoint = pytest.importorskip("paper_2607_04516_amd.adjoint")


def _setup(storage, steps, every, small=True, nx=64, ny=64, nz=32):
    w = workloads.adjoint_urban(storage, steps, small=small)
    lat = binding.from_workload(w)
    base = workloads.power_law_speeds(w.nz, 0.08, 100.0 if not small else 25.0, 0.25)
    prob = adjoint.InflowProblem(lat, w.probes, steps, every, w.u0)
    return w, lat, prob, base


def _target(prob, base, seed=12):
    rng = np.random.default_rng(seed)
    sp = base * (1 + 0.05 * rng.uniform(-1, 1, base.shape))
    ub, _ = prob.run_forward(sp, math.radians(5.0), keep_checkpoints=False)
    return ub


def _loss_grad(prob, speeds, theta, target):
    s = torch.tensor(speeds, dtype=torch.float64, requires_grad=True)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    L = adjoint.probe_misfit(prob, s, th, target)
    L.backward()
    return float(L), np.concatenate([s.grad.numpy(), [float(th.grad)]])


def _fd(prob, speeds, theta, target, h=1e-4, comps=None):
    n = len(speeds) + 1
    comps = range(n) if comps is None else comps
    out = {}
    for k in comps:
        vals = []
        for sgn in (1, -1):
            sp, th = speeds.copy(), theta
            if k < len(speeds):
                sp[k] += sgn * h
            else:
                th += sgn * h
            ub, _ = prob.run_forward(sp, th, keep_checkpoints=False)
            vals.append(float(((ub - target) ** 2).sum()))
        out[k] = (vals[0] - vals[1]) / (2 * h)
    return out


def test_gradient_f64_matches_central_differences():
    print("case: adjoint 64x64x32 f64, T=200, K=25, all 33 parameters", flush=True)
    w, lat, prob, base = _setup("f64", 200, 25)
    target = _target(prob, base)
    L, g = _loss_grad(prob, base.copy(), 0.0, target)
    fd = _fd(prob, base.copy(), 0.0, target)
    gfd = np.array([fd[k] for k in range(len(g))])
    rel = np.linalg.norm(g - gfd) / np.linalg.norm(gfd)
    print(f"loss {L:.4e}  |g| {np.linalg.norm(g):.4e}  rel err vs FD {rel:.2e}", flush=True)
    assert rel <= 1e-3


def test_gradient_f32_adjoint_within_1e3_of_fd():
    print("case: adjoint 64x64x32 f32 vs f64 FD, T=200, K=50", flush=True)
    w, lat, prob, base = _setup("f64", 200, 50)
    target = _target(prob, base)
    fd = _fd(prob, base.copy(), 0.0, target)
    gfd = np.array([fd[k] for k in range(len(fd))])
    w32, lat32, prob32, _ = _setup("f32", 200, 50)
    L, g = _loss_grad(prob32, base.copy(), 0.0, target.float().double())
    rel = np.linalg.norm(g - gfd) / np.linalg.norm(gfd)
    print(f"f32 adjoint vs f64 FD: rel err {rel:.2e}", flush=True)
    assert rel <= 1e-3


def test_gradient_matches_cpu_oracle_adjoint():
    """FP64 GPU gradient against the oracle's FP64 scatter-transpose adjoint."""
    nx, ny, nz, T = 24, 16, 12, 30
    h = workloads.urban_heights(nx, ny, 0.3, 4, 0.5, 8, 5, footprint=(2, 5), margin_x=6, margin_y=2)
    solid = workloads.heights_to_mask(h, nz)
    probes = workloads.probe_cells(h, nz, 6, 9, margin_x=6, margin_y=2)
    prof = workloads.direction_profile(workloads.power_law_speeds(nz, 0.06, 8.0, 0.25), 0.0)
    w = workloads.Workload("tiny", nx, ny, nz, workloads.FACES_CHANNEL, 0.53, 0.1, "f64", T, solid,
                           {0: prof}, prof.copy(), noise_seed=3, probes=probes)
    lat = binding.from_workload(w)
    prob = adjoint.InflowProblem(lat, probes, T, 10, w.u0)
    speeds = prof[:, 0].copy()
    theta = 0.05
    target = torch.zeros(len(probes), 3, dtype=torch.float64)
    target[:, 0] = 0.05
    L, g = _loss_grad(prob, speeds, theta, target)

    # oracle: same forward, FP64 scatter-transpose adjoint
    o = oracle_for(w)
    o.inflow[0] = prob.profile(speeds, theta)
    f = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
    traj = [f]
    ubar = np.zeros((len(probes), 3))
    for t in range(T):
        f = o.step(f)
        traj.append(f)
        _, u, _ = o.macros(f)
        ubar += np.array([u[:, z, y, x] for x, y, z in probes])
    ubar /= T
    src = 2 * (ubar - target.numpy()) / T
    lam = np.zeros_like(f)
    gsum = np.zeros((6, nz, 3))
    for t in range(T, -1, -1):
        lam, gg = o.adjoint_step(traj[t], lam, probes, src if t >= 1 else None)
        gsum += gg
    gp = gsum[0]
    d_sp = gp[:, 0] * math.cos(theta) + gp[:, 1] * math.sin(theta)
    d_th = float((gp[:, 0] * (-speeds * math.sin(theta)) + gp[:, 1] * speeds * math.cos(theta)).sum())
    go = np.concatenate([d_sp, [d_th]])
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"GPU vs oracle adjoint gradient: rel {rel:.2e}", flush=True)
    assert rel <= 1e-10


def test_push_chain_reproduces_forward_bit_exact():
    """The recompute (out-of-place push steps) reproduces the in-place run."""
    w = workloads.adjoint_urban("f32", 20, small=True)
    lat = binding.from_workload(w)
    s0, _ = lat.get_state()
    s0 = s0.clone()
    lat.step(20)
    ref, _ = lat.get_state()
    a, b = s0.clone(), lat.new_state()
    for _ in range(20):
        lat.push_step(a, b)
        a, b = b, a
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
