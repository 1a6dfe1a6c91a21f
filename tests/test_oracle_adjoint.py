"""Pins of the oracle's discrete adjoint (FP64, CPU).

The adjoint is pinned by central finite differences of the oracle's own
forward map, which is itself pinned in test_oracle_pins.py:
  * the explicit collision Jacobian against differences of or_collide;
  * the one-step transpose (dot-product) identity <lam, J v> = <J^T lam, v>
    with J v by central differences, including the inflow-profile part;
  * the gradient of a time-averaged probe-velocity misfit with respect to
    per-height inflow speeds and the inflow angle against central
    differences of the whole run.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import fluid_mask, oracle_for, small_workload
from paper_2607_04516_amd import workloads


def _cell(seed, rho=1.01, u=(0.04, -0.02, 0.03), amp=0.03):
    rng = np.random.default_rng(seed)
    return oracle.equilibrium(rho, u) * (1.0 + amp * (rng.random(19) - 0.5))


@pytest.mark.parametrize("omega", [(0.0, 0.0, 0.0), (0.0, 2e-3, 4e-3)])
@pytest.mark.parametrize("force", [(0.0, 0.0, 0.0), (3e-4, -1e-4, 2e-4)])
@pytest.mark.parametrize("c_smag", [0.0, 0.1, 0.3])
def test_jacobian_matches_central_differences(force, c_smag, omega):
    o = oracle.Oracle(3, 3, 3, [oracle.PERIODIC] * 6, tau0=0.52, c_smag=c_smag, force=force, omega=omega)
    for seed in range(3):
        f = _cell(seed)
        J = o.collide_jacobian(f)
        h = 1e-6
        Jfd = np.zeros((19, 19))
        for j in range(19):
            e = np.zeros(19)
            e[j] = h
            Jfd[:, j] = (o.collide(f + e)[0] - o.collide(f - e)[0]) / (2 * h)
        assert np.abs(J - Jfd).max() <= 1e-8 * max(1.0, np.abs(J).max())


def _step_problem(faces, seed=0):
    nx, ny, nz = 9, 7, 6
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8)
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.15, u=(0.05, 0.02, 0.0),
                       noise=5e-3, seed=seed + 3)
    o = oracle_for(w)
    f = o.run(o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed), 4)
    return w, o, f, rng


@pytest.mark.parametrize("faces", [
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
    ("periodic", "periodic", "wall", "outflow", "freeslip", "outflow"),
])
def test_step_transpose_dot_product(faces):
    w, o, f, rng = _step_problem(faces)
    m = fluid_mask(w)
    v = rng.standard_normal(f.shape) * m[None]
    lam_next = rng.standard_normal(f.shape) * m[None]
    eps = 1e-7
    jv = (o.step(f + eps * v) - o.step(f - eps * v)) / (2 * eps)
    lam, g = o.adjoint_step(f, lam_next)
    lhs = float((lam_next * jv * m[None]).sum())
    rhs = float((lam * v).sum())
    assert abs(lhs - rhs) <= 1e-7 * abs(lhs)
    # inflow-profile part: d step / d u_in . du against g . du
    du = rng.standard_normal((6, w.nz, 3))
    for k in range(6):
        if faces[k] != "inflow":
            du[k] = 0.0
    base = o.inflow.copy()
    o.inflow[:] = base + eps * du
    fp = o.step(f)
    o.inflow[:] = base - eps * du
    fm = o.step(f)
    o.inflow[:] = base
    lhs = float((lam_next * (fp - fm) / (2 * eps) * m[None]).sum())
    rhs = float((g * du).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def _loss_and_grad(o, w, speeds, theta, probes, target, T, with_grad=True):
    """Loss sum_p |mean_{t=1..T} u(x_p, t) - target_p|^2 with the x- inflow
    profile speeds[z] (cos theta, sin theta, 0); gradient by the oracle adjoint."""
    prof = np.stack([speeds * math.cos(theta), speeds * math.sin(theta), np.zeros_like(speeds)], 1)
    o.inflow[0] = prof
    f0 = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
    traj = [f0]
    ubar = np.zeros((len(probes), 3))
    f = f0
    for t in range(T):
        f = o.step(f)
        traj.append(f)
        _, u, _ = o.macros(f)
        ubar += np.array([u[:, z, y, x] for x, y, z in probes])
    ubar /= T
    loss = float(((ubar - target) ** 2).sum())
    if not with_grad:
        return loss, None
    src = 2.0 * (ubar - target) / T
    lam = np.zeros_like(f0)
    gsum = np.zeros((6, w.nz, 3))
    for t in range(T, -1, -1):
        lam, g = o.adjoint_step(traj[t], lam, probes, src if t >= 1 else None)
        gsum += g
    gp = gsum[0]
    d_speeds = gp[:, 0] * math.cos(theta) + gp[:, 1] * math.sin(theta)
    d_theta = float((gp[:, 0] * (-speeds * math.sin(theta)) + gp[:, 1] * speeds * math.cos(theta)).sum())
    return loss, np.concatenate([d_speeds, [d_theta]])


@pytest.mark.parametrize("omega", [(0.0, 0.0, 0.0), (0.0, 3e-3, 6e-3)])
def test_full_gradient_matches_finite_differences(omega):
    nx, ny, nz, T = 14, 8, 6, 12
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0:3, 3:5, 6:8] = 1
    w = small_workload(nx, ny, nz, ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
                       solid=solid, tau0=0.55, c_smag=0.15, u=(0.05, 0.0, 0.0), noise=1e-3, seed=2,
                       omega=omega)
    o = oracle_for(w)
    probes = np.array([[9, 4, 4], [7, 2, 3], [11, 6, 1]], np.int32)
    speeds = workloads.power_law_speeds(nz, 0.05, 4.0, 0.25)
    theta = 0.1
    target = np.zeros((3, 3))
    target[:, 0] = 0.045
    loss, grad = _loss_and_grad(o, w, speeds, theta, probes, target, T)
    h = 1e-6
    fd = np.zeros(nz + 1)
    for k in range(nz + 1):
        sp, tp = speeds.copy(), theta
        sm, tm = speeds.copy(), theta
        if k < nz:
            sp[k] += h
            sm[k] -= h
        else:
            tp += h
            tm -= h
        fd[k] = (_loss_and_grad(o, w, sp, tp, probes, target, T, False)[0]
                 - _loss_and_grad(o, w, sm, tm, probes, target, T, False)[0]) / (2 * h)
    assert np.linalg.norm(grad - fd) <= 1e-6 * np.linalg.norm(fd)
