"""Write the oracle's reference gradient for the adjoint workload's 64x64x32 copy.

Loss (time-averaged probe misfit): L = sum_p |u_bar_p - target_p|^2 with
u_bar_p = (1/T) sum_{t=1..T} u(x_p, t), T = 1000, 24 probe cells; the
parameters are the 32 per-height speeds s_k of the x- inflow face and the
inflow angle theta, u_in(k) = s_k (cos theta, sin theta, 0), at the base
point s = power law (u_ref 0.08 at z_ref 25, alpha 0.25), theta = 0.  The
targets are the oracle's own u_bar for speeds s (1 + 0.05 xi_k), xi ~ U(-1, 1)
(numpy PCG64, seed 12), and theta = 5 degrees.  The initial state is the
workload's (base profile plus seeded noise) and is not differentiated.

Everything here is computed by the FP64 CPU oracle only (forward steps and
its scatter-transpose discrete adjoint, with the trajectory recomputed from
checkpoints every 50 steps); the inputs come from the seeded workload
generator.  Output: adjoint_copy_64x64x32_T1000.json next to this script.
Run time is about 20 minutes on one core.

    python tests/golden/make_adjoint_copy_golden.py
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_04516_amd import workloads  # noqa: E402

T, K = 1000, 50
OUT = os.path.join(HERE, "adjoint_copy_64x64x32_T1000.json")
FACE_NUM = {"periodic": oracle.PERIODIC, "inflow": oracle.INFLOW_EQ, "outflow": oracle.OUTFLOW_ZG,
            "freeslip": oracle.FREESLIP, "wall": oracle.WALL}


def profile(speeds, theta):
    s = np.asarray(speeds, np.float64)
    return np.stack([s * math.cos(theta), s * math.sin(theta), np.zeros_like(s)], axis=1)


def make_oracle(w):
    return oracle.Oracle(w.nx, w.ny, w.nz, [FACE_NUM[f] for f in w.faces], tau0=w.tau0, c_smag=w.c_smag,
                         delta=w.delta, solid=w.solid, inflow={0: w.inflow[0]})


def forward(o, w, speeds, theta, keep_every=0):
    """u_bar over t = 1..T and, with keep_every, the states at t = 0, K, 2K, ..."""
    o.inflow[0] = profile(speeds, theta)
    f = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
    pr = np.asarray(w.probes)
    ubar = np.zeros((len(pr), 3))
    ckpts = []
    for t in range(T):
        if keep_every and t % keep_every == 0:
            ckpts.append(f.copy())
        f = o.step(f)
        _, u, _ = o.macros(f)
        ubar += u[:, pr[:, 2], pr[:, 1], pr[:, 0]].T
    return ubar / T, ckpts


def main():
    t_start = time.time()
    w = workloads.adjoint_urban("f64", T, small=True)
    o = make_oracle(w)
    base = workloads.power_law_speeds(w.nz, 0.08, 25.0, 0.25)
    rng = np.random.default_rng(12)
    sp_t = base * (1 + 0.05 * rng.uniform(-1, 1, base.shape))
    target, _ = forward(o, w, sp_t, math.radians(5.0))
    print(f"target run done ({time.time() - t_start:.0f} s)", flush=True)
    theta = 0.0
    ubar, ckpts = forward(o, w, base, theta, keep_every=K)
    loss = float(((ubar - target) ** 2).sum())
    print(f"base run done ({time.time() - t_start:.0f} s), loss {loss:.6e}", flush=True)
    src = 2.0 * (ubar - target) / T
    pr = np.asarray(w.probes, np.int32)
    o.inflow[0] = profile(base, theta)
    lam = np.zeros((19, w.nz, w.ny, w.nx))
    gsum = np.zeros((6, w.nz, 3))
    for seg in range(T // K - 1, -1, -1):
        traj = [ckpts[seg]]
        for _ in range(K):
            traj.append(o.step(traj[-1]))
        first = 0 if seg == 0 else seg * K + 1
        for t in range(seg * K + K, first - 1, -1):
            lam, g = o.adjoint_step(traj[t - seg * K], lam, pr, src if t >= 1 else None)
            gsum += g
        print(f"segment {seg} done ({time.time() - t_start:.0f} s)", flush=True)
    gp = gsum[0]
    c, s = math.cos(theta), math.sin(theta)
    d_sp = gp[:, 0] * c + gp[:, 1] * s
    d_th = float((gp[:, 0] * (-base * s) + gp[:, 1] * (base * c)).sum())
    rec = {
        "what": "oracle FP64 gradient of L = sum_p |u_bar_p - target_p|^2 (T = 1000, checkpoints every 50) "
                "for the adjoint workload's 64x64x32 copy; written by make_adjoint_copy_golden.py from oracle/ only",
        "T": T, "K": K, "theta": theta, "speeds": base.tolist(),
        "target_speeds": sp_t.tolist(), "target_theta_deg": 5.0,
        "target": target.tolist(), "ubar": ubar.tolist(), "loss": loss,
        "grad_speeds": d_sp.tolist(), "grad_theta": d_th,
        "seconds": round(time.time() - t_start, 1),
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {OUT}: |g| {np.linalg.norm(np.append(d_sp, d_th)):.6e}", flush=True)


if __name__ == "__main__":
    main()
