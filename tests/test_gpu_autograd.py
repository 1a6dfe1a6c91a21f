"""Checkpointed discrete adjoint behind torch.autograd.Function (needs an MI355X).

Loss: sum over probes of |time-averaged u - target|^2, parameters: the
per-height inflow speeds of the x- face and the inflow angle.  Checked
against central finite differences (h = 1e-4) of the FP64 GPU forward, and
against the FP64 CPU oracle adjoint: over the adjoint workload's 64x64x32
copy at its full length (T = 1000, checkpoints every 50; the oracle's
gradient and targets in tests/golden/, written by a script that calls only
the oracle), over a short trajectory on a tiny grid, and on the full
256x256x96 grid for a sample of parameters.  Every gradient component is
checked on its own (relative bar plus a stated absolute floor), the angle
separately.
"""
import json
import math
import os

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
            vals.append(float(((ub - target.to(ub.device, ub.dtype)) ** 2).sum()))
        out[k] = (vals[0] - vals[1]) / (2 * h)
    return out


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


# --------------------------------------------------------------------------
# The adjoint workload's 64x64x32 copy at its full length: T = 1000, K = 50.
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_copy_64x64x32_T1000.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _copy_problem(storage):
    gd = _golden()
    w, lat, prob, base = _setup(storage, gd["T"], gd["K"])
    assert np.array_equal(np.asarray(gd["speeds"]), base)
    target = torch.tensor(gd["target"], dtype=torch.float64)
    return gd, prob, base, target


def _per_component(g, ref, rel, floor, what):
    """|g_k - ref_k| <= rel |ref_k| + floor for every k; prints the worst."""
    err = np.abs(g - ref)
    lim = rel * np.abs(ref) + floor
    k = int(np.argmax(err / lim))
    print(f"{what}: worst component {k}: |d| {err[k]:.3e} vs bar {lim[k]:.3e} (ref {ref[k]:.3e}); "
          f"angle |d| {err[-1]:.3e} of {abs(ref[-1]):.3e}; norm rel {np.linalg.norm(err) / np.linalg.norm(ref):.2e}",
          flush=True)
    assert np.all(err <= lim), (what, np.nonzero(err > lim)[0].tolist())


@pytest.fixture(scope="module")
def copy_fd():
    """Central differences (h = 1e-4) of the FP64 GPU forward at T = 1000 for
    all 33 parameters of the copy, and its FP64 adjoint gradient."""
    print("case: adjoint copy 64x64x32 f64, T=1000, K=50: FD over 33 parameters", flush=True)
    gd, prob, base, target = _copy_problem("f64")
    L, g = _loss_grad(prob, base.copy(), 0.0, target)
    fd = _fd(prob, base.copy(), 0.0, target)
    return gd, L, g, np.array([fd[k] for k in range(len(g))])


def test_copy_f64_gradient_matches_oracle_adjoint(copy_fd):
    """FP64 GPU gradient (T = 1000, K = 50) against the oracle's FP64
    scatter-transpose adjoint, with the oracle's own targets."""
    gd, L, g, _ = copy_fd
    go = np.array(gd["grad_speeds"] + [gd["grad_theta"]])
    print(f"loss gpu {L:.10e} oracle {gd['loss']:.10e}", flush=True)
    assert abs(L - gd["loss"]) <= 1e-10 * gd["loss"]
    _per_component(g, go, 1e-8, 1e-10 * np.abs(go).max(), "f64 gpu vs oracle adjoint")
    assert np.linalg.norm(g - go) <= 1e-10 * np.linalg.norm(go)


def test_copy_f64_gradient_matches_central_differences(copy_fd):
    """FP64 adjoint against central differences: per component within
    1e-4 relative plus 1e-6 of the largest component (the O(h^2) truncation
    of the differences), and 1e-3 in norm."""
    _, _, g, gfd = copy_fd
    _per_component(g, gfd, 1e-4, 1e-6 * np.abs(gfd).max(), "f64 adjoint vs FD")
    assert np.linalg.norm(g - gfd) <= 1e-3 * np.linalg.norm(gfd)


def test_copy_f32_adjoint_matches_central_differences(copy_fd):
    """FP32 forward, recompute and adjoint against the FP64 central
    differences: 1e-3 in norm; per component within 1e-2 relative plus 1e-3
    of the largest component (the FP32 trajectory's own rounding)."""
    gd, _, _, gfd = copy_fd
    _, prob32, base, target = _copy_problem("f32")
    L, g = _loss_grad(prob32, base.copy(), 0.0, target.float().double())
    _per_component(g, gfd, 1e-2, 1e-3 * np.abs(gfd).max(), "f32 adjoint vs f64 FD")
    assert np.linalg.norm(g - gfd) <= 1e-3 * np.linalg.norm(gfd)


def test_full_grid_f32_gradient_matches_central_differences():
    """The 256x256x96 adjoint workload itself (T = 1000, K = 50): the FP32
    adjoint gradient against central differences (h = 1e-4) of the FP64
    forward for the angle and seven speeds spread over the height."""
    print("case: adjoint 256x256x96 f32 T=1000 K=50 vs f64 FD (8 parameters)", flush=True)
    w64, lat64, prob64, base = _setup("f64", 1000, 50, small=False)
    target = _target(prob64, base)
    comps = [0, 5, 15, 30, 50, 75, 95, 96]
    fd = _fd(prob64, base.copy(), 0.0, target, comps=comps)
    lat64.close()
    _, _, prob32, _ = _setup("f32", 1000, 50, small=False)
    L, g = _loss_grad(prob32, base.copy(), 0.0, target.float().double())
    gs, fs = g[comps], np.array([fd[k] for k in comps])
    full = np.abs(g).max()
    for k, a, b in zip(comps, gs, fs):
        print(f"  param {k}: adjoint {a:.6e} FD {b:.6e}", flush=True)
    err = np.abs(gs - fs)
    assert np.all(err <= 1e-2 * np.abs(fs) + 1e-3 * full), err
    assert np.linalg.norm(err) <= 1e-3 * np.linalg.norm(fs) + 1e-3 * full
