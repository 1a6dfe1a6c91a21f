#!/usr/bin/env python3
"""Benchmark of the fused D3Q19 LBM-LES step on one MI355X.

Workload: the kilometre-scale urban analogue, 800 x 800 x 128 cells (81.9M),
buildings at plan-area fraction 0.30 (median height 12 cells), power-law
inflow (alpha 0.22, 0.08 at z = 100) at 30 degrees on the x- and y- faces,
zero-gradient outflow on x+ and y+, bounce-back ground, free-slip top,
tau0 = 0.505, C = 0.1, FP32 storage.  Inputs are seeded and synthetic and
sit in HBM before the timed region.

Prints ONE JSON line: MLUPS (fluid-cell updates per second) of the FP32
forward step, the step kernel's achieved HBM bandwidth against the 8 TB/s
peak from HIP events around every launch in the timed region, the shifted
binary16 / bfloat16 storage rates, and the FP64 CPU oracle timed on a
bounded crop of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + achieved HBM GB/s (fwd FP32 vs FP16-storage; adjoint), 1 MI355X"
HBM_PEAK_GBS = 8000.0
NQ = 19
STORE_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}


def algorithmic_bytes(lat, storage):
    """Bytes one step-kernel launch must move: interior fluid cells read and
    write 19 populations, inflow cells write 19, solid cells nothing (the
    solid-mask bits, N/8 bytes, are negligible and not counted)."""
    fluid, interior = lat.cell_counts()
    b = STORE_BYTES[storage]
    return interior * 2 * NQ * b + (fluid - interior) * NQ * b


def time_forward(w, storage, steps, warmup, setup=None):
    import torch

    from paper_2607_04516_amd import binding
    lat = binding.from_workload(w, storage=storage)
    if setup is not None:
        setup(lat)
    lat.step(warmup)
    torch.cuda.synchronize()
    lat.profile(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    lat.step(steps)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    kern_ms, launches = lat.profile_read()
    lat.profile(False)
    fluid, _ = lat.cell_counts()
    rows, nyp, pitch = lat.layout()
    mlups = fluid * steps / (ms * 1e-3) / 1e6
    per_launch_ms = kern_ms / max(launches, 1)
    bytes_launch = algorithmic_bytes(lat, storage)
    gbs = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    # sanity: the run stayed finite
    m, e = lat.mass()
    lat.close()
    return {"mlups": mlups, "ms_per_step": ms / steps, "kernel_ms": per_launch_ms, "launches": launches,
            "bytes_per_launch": bytes_launch, "achieved_gbs": gbs, "fluid_cells": fluid,
            "mass": m, "energy": e,
            "layout": f"row blocks [{nyp}*nz/{rows}][19][{rows} rows][{pitch}], in-place A-A"}


def time_adjoint(steps=1000, every=50):
    """Adjoint workload: 256 x 256 x 96 urban grid, FP32, T steps with a
    checkpoint every K; loss = sum over 24 probes of |u_bar - target|^2,
    gradient with respect to 96 inflow speeds and the angle.  Returns the
    plain-forward, checkpointed-forward and backward times."""
    import math

    import numpy as np
    import torch

    from paper_2607_04516_amd import adjoint, binding, workloads
    w = workloads.adjoint_urban("f32", steps)
    lat = binding.from_workload(w)
    base = workloads.power_law_speeds(w.nz, 0.08, 100.0, 0.25)
    prob = adjoint.InflowProblem(lat, w.probes, steps, every, w.u0)
    rng = np.random.default_rng(12)
    tgt, _ = prob.run_forward(base * (1 + 0.05 * rng.uniform(-1, 1, base.shape)), math.radians(5.0),
                              keep_checkpoints=False)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # plain forward: T steps, nothing else
    lat.reset(w.u0)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    lat.step(steps)
    b.record()
    torch.cuda.synchronize()
    t_plain = a.elapsed_time(b)
    sp = torch.tensor(base, dtype=torch.float64, requires_grad=True)
    th = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = adjoint.probe_misfit(prob, sp, th, tgt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fluid, _ = lat.cell_counts()
    g = np.concatenate([sp.grad.numpy(), [float(th.grad)]])
    lat.close()
    return {"workload": f"{w.name}, FP32, T={steps}, K={every}, {len(w.probes)} probes, 97 parameters",
            "forward_plain_ms": round(t_plain, 2), "forward_ckpt_ms": round((t1 - t0) * 1e3, 2),
            "backward_ms": round((t2 - t1) * 1e3, 2),
            "cost_ratio": round(((t1 - t0) + (t2 - t1)) * 1e3 / t_plain, 3),
            "adjoint_mlups": round(fluid * steps / (t2 - t1) / 1e6, 1),
            "loss": float(L), "grad_norm": float(np.linalg.norm(g))}


def adjoint_child(steps):
    """time_adjoint in a fresh process (bench.py --adjoint-only); its record."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--adjoint-only", "--adjoint-steps", str(steps)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"adjoint child process failed with status {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])["adjoint"]


def time_shard(w, n=8, steps=40, warmup=4):
    """The kilometre grid as n slabs along y (one per rank of an n-GPU run),
    all on this GPU: every slab steps, then the halo exchange runs (the five
    crossing populations per interface and direction).  Returns the time per
    step of all slabs together and of one slab's share, the exchange part,
    the halo bytes, and whether the slabs match the whole-grid run bit for
    bit after the timed steps."""
    import torch

    from paper_2607_04516_amd import binding, slabs
    whole = binding.from_workload(w)
    dec = slabs.SlabDecomposition(w, n)
    s0, _ = whole.get_state()
    dec.set_state(s0, 0)
    del s0
    dec.step(warmup)
    whole.step(warmup)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t_step = t_exch = 0.0
    for _ in range(steps):
        a, b, c = ev(), ev(), ev()
        a.record()
        for lat in dec.slabs:
            lat.step(1)
        b.record()
        dec.exchange()
        c.record()
        torch.cuda.synchronize()
        t_step += a.elapsed_time(b)
        t_exch += a.elapsed_time(c) - a.elapsed_time(b)
    whole.step(steps)
    ref, _ = whole.get_state()
    same = bool(torch.equal(dec.get_state(), ref))
    rows = [y1 - y0 for y0, y1 in dec.rows]
    b = torch.empty(0, dtype=dec.slabs[0].store_dtype).element_size()
    dec.close()
    whole.close()
    per = (t_step + t_exch) / steps
    return {"slabs": n, "rows_per_slab": rows[0], "ms_per_step_all_slabs": round(per, 4),
            "ms_per_step_per_slab": round(per / n, 4), "exchange_ms_per_step_all_slabs": round(t_exch / steps, 4),
            "halo_bytes_per_interface_per_step": 2 * 5 * w.nx * w.nz * b,
            "bit_identical_to_whole_grid": same}


def time_voxelize(nx=800, ny=800, nz=128):
    """Voxelize the kilometre workload's buildings (box meshes from the same
    draws as its height map) with 1 and 3 ray directions; wall time of the
    call (host input and output included) and whether the mask equals the
    height-map mask."""
    from paper_2607_04516_amd import binding, workloads
    meshes = workloads.urban_box_meshes(nx, ny, 0.30, 12, 0.5, 100, 5, (10, 40), 32, 32)
    t, s = workloads.meshes_to_arrays(meshes)
    want = workloads.heights_to_mask(workloads.urban_heights(nx, ny, 0.30, 12, 0.5, 100, 5, (10, 40), 32, 32), nz)
    out = {"meshes": len(meshes), "triangles": int(len(t)), "cells": nx * ny * nz}
    for passes in (1, 3):
        binding.voxelize((nz, ny, nx), t, s, passes)          # warm-up
        t0 = time.perf_counter()
        got = binding.voxelize((nz, ny, nx), t, s, passes)
        out[f"ms_{passes}_pass"] = round((time.perf_counter() - t0) * 1e3, 2)
        out[f"equals_height_map_{passes}_pass"] = bool((got == want).all())
    return out


FEATURE_NAMES = ("coriolis", "von_karman_inflow", "sponge", "flux_balance_every_step")


def apply_feature(lat, name):
    """The paper's additions to the step (App. E, App. F, Sec. 2.2), on the bench grid."""
    from paper_2607_04516_amd import binding
    if name == "coriolis":            # Earth rotation at 23.113 N, dt = 0.01 s
        lat.set_rotation(binding.earth_rotation(23.113, 0.01))
    elif name == "von_karman_inflow":  # 64 modes per face, L = 20 cells, 10% intensity
        lat.set_turbulence(n_modes=64, length_scale=20.0, intensity=0.1, seed=1)
    elif name == "sponge":             # 16-cell layers next to the inflow faces
        lat.set_sponge(16, 0.05)
    elif name == "flux_balance_every_step":
        lat.balance_flux(2)
    else:
        raise ValueError(name)


def time_features(w, steps, warmup):
    """FP32 step rate with each source or stabiliser switched on alone, and
    all together; and with the mean/RMS velocity statistics accumulated
    every 10 steps (the long-run statistics of Sec. 2.3)."""
    import torch
    out = {}
    for name in FEATURE_NAMES + ("all",):
        def setup(lat, name=name):
            for k in (FEATURE_NAMES if name == "all" else (name,)):
                apply_feature(lat, k)
        r = time_forward(w, "f32", steps, warmup, setup)
        out[name] = {"value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 4)}
    acc = torch.zeros(6, w.nz, w.ny, w.nx, dtype=torch.float32, device="cuda")
    r = time_forward(w, "f32", steps, warmup, lambda lat: lat.set_stats(acc, 10))
    out["stats_every_10_steps"] = {"value": round(r["mlups"], 1), "unit": "MLUPS",
                                   "ms_per_step": round(r["ms_per_step"], 4)}
    del acc
    torch.cuda.empty_cache()
    return out


def copy_bandwidth():
    """Device-to-device copy of 4 GiB, best of 5: an achievable HBM figure on this machine."""
    import torch
    a = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


# the files that define the step kernels k_even / k_odd (the counter record
# stays valid while these are unchanged)
STEP_KERNEL_SOURCES = ("lbm_step.hip", "lbm_device.h", "lbm_launch.h", "lbm_general.h")


def traffic_from_profiles(storage, workload):
    """HBM bytes per step-kernel launch from the committed counter summary,
    if it was taken on this workload and the current kernel sources (else
    None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_even_k_odd_urban_km_800x800x128.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2607_04516_amd", "csrc")
    for f in STEP_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    if (rec.get("sources_sha256") != h.hexdigest() or rec.get("workload") != workload
            or storage not in rec.get("per_launch_bytes", {})):
        return None, rec.get("sources_sha256")
    return rec["per_launch_bytes"][storage], rec.get("sources_sha256")


def traffic_request_sizes(storage, workload):
    """The same per-launch bytes counted a second way (L2 -> memory read
    requests weighted by their size, 32/64/128 B, plus write requests of 64
    and 32 B), from the same summary; None when stale or absent."""
    tb, sha = traffic_from_profiles(storage, workload)
    if tb is None:
        return None
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_even_k_odd_urban_km_800x800x128.json")))
    return rec.get("per_launch_bytes_request_sizes", {}).get(storage)


def cpu_info():
    """(CPU model name, cores this process may use, logical CPUs of the host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, usable, os.cpu_count()


def cpu_baseline_openmp(seconds=12.0, crop=(160, 160)):
    """The same oracle source built with OpenMP over the step's z planes
    (oracle variant "omp"), timed in a child process on the cores this
    process may use (OMP_NUM_THREADS if set)."""
    import subprocess
    _, usable, _ = cpu_info()
    env = dict(os.environ, LBM_ORACLE_VARIANT="omp")
    env.setdefault("OMP_NUM_THREADS", str(usable))
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--cpu-omp-only", "--cpu-crop", str(crop[0]), str(crop[1]),
           "--cpu-seconds", str(seconds)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600, env=env)
    if r.returncode != 0:
        raise RuntimeError(f"OpenMP oracle child failed with status {r.returncode}")
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    rec["cores"] = int(env["OMP_NUM_THREADS"])
    return rec


def cpu_baseline(w, seconds=12.0, crop=(160, 160)):
    """The FP64 oracle (single thread) on a crop of the workload: the first
    crop[0] x crop[1] columns with the full height, same faces and profiles."""
    import numpy as np

    import oracle
    from paper_2607_04516_amd import workloads

    cx, cy = crop
    solid = np.ascontiguousarray(w.solid[:, :cy, :cx])
    faces = {"periodic": oracle.PERIODIC, "inflow": oracle.INFLOW_EQ, "outflow": oracle.OUTFLOW_ZG,
             "freeslip": oracle.FREESLIP, "wall": oracle.WALL}
    o = oracle.Oracle(cx, cy, w.nz, [faces[f] for f in w.faces], tau0=w.tau0, c_smag=w.c_smag,
                      solid=solid, inflow=w.inflow)
    f = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
    fluid = int(solid.size - np.count_nonzero(solid))
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = o.step(f)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    threads = os.environ.get("OMP_NUM_THREADS", "1") if os.environ.get("LBM_ORACLE_VARIANT") == "omp" else "1"
    model, usable, logical = cpu_info()
    return {"value": fluid * steps / el / 1e6, "unit": "MLUPS", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 oracle, {threads} thread(s), {cx}x{cy}x{w.nz} crop of {w.name} "
                      f"({fluid} fluid cells), {steps} steps in {el:.1f} s",
            "cpu_model": model, "nproc": usable, "logical_cpus": logical}


def oracle_configs(adjoint_steps=50):
    """The FP64 oracle (single thread) on the configurations small enough to
    run whole: the 64x48x32 cube flow and the 128x128x64 urban subdomain for
    100 steps each, and the adjoint copy (64x64x32): adjoint_steps forward
    steps from the initial state, then as many adjoint steps back over the
    stored trajectory.  Opt-in (--oracle-configs): about two minutes."""
    import numpy as np

    import oracle
    from paper_2607_04516_amd import workloads
    faces = {"periodic": oracle.PERIODIC, "inflow": oracle.INFLOW_EQ, "outflow": oracle.OUTFLOW_ZG,
             "freeslip": oracle.FREESLIP, "wall": oracle.WALL}

    def make(w):
        return oracle.Oracle(w.nx, w.ny, w.nz, [faces[f] for f in w.faces], tau0=w.tau0, c_smag=w.c_smag,
                             delta=w.delta, solid=w.solid, inflow=w.inflow, force=w.force)

    def fluid(w):
        return int(w.solid.size - np.count_nonzero(w.solid))

    out = {}
    for key, w in (("cube_64x48x32", workloads.cube_flow("f64", 100)),
                   ("urban_subdomain_128x128x64", workloads.urban_subdomain("f64", 100))):
        o = make(w)
        f = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
        t0 = time.perf_counter()
        for _ in range(100):
            f = o.step(f)
        el = time.perf_counter() - t0
        out[key] = {"steps": 100, "seconds": round(el, 2), "mlups": round(fluid(w) * 100 / el / 1e6, 3)}
    w = workloads.adjoint_urban("f64", adjoint_steps, small=True)
    o = make(w)
    f = o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)
    pr = np.asarray(w.probes, np.int32)
    traj = [f]
    t0 = time.perf_counter()
    for _ in range(adjoint_steps):
        traj.append(o.step(traj[-1]))
    t_fwd = time.perf_counter() - t0
    src = np.full((len(pr), 3), 1.0 / adjoint_steps)
    lam = np.zeros((19, w.nz, w.ny, w.nx))
    t0 = time.perf_counter()
    for t in range(adjoint_steps, 0, -1):
        lam, _ = o.adjoint_step(traj[t], lam, pr, src)
    t_adj = time.perf_counter() - t0
    n = fluid(w) * adjoint_steps / 1e6
    out["adjoint_copy_64x64x32"] = {"steps": adjoint_steps, "forward_seconds": round(t_fwd, 2),
                                    "adjoint_seconds": round(t_adj, 2), "forward_mlups": round(n / t_fwd, 3),
                                    "adjoint_mlups": round(n / t_adj, 3),
                                    "adjoint_over_forward": round(t_adj / t_fwd, 2)}
    model, usable, logical = cpu_info()
    return {"kind": "oracle", "threads": 1, "cpu_model": model, "nproc": usable, "logical_cpus": logical,
            "configs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 16-bit storage runs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-cost run")
    ap.add_argument("--no-features", action="store_true", help="skip the Coriolis / inflow / stabiliser runs")
    ap.add_argument("--no-shard", action="store_true", help="skip the 8-slab decomposition run")
    ap.add_argument("--no-voxelize", action="store_true", help="skip the voxelizer run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 2 GiB device buffer three times: the known-size kernel that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint-cost workload and print its record (for profiling)")
    ap.add_argument("--adjoint-steps", type=int, default=1000, help="time steps T of the adjoint workload")
    ap.add_argument("--oracle-configs", action="store_true",
                    help="time the FP64 oracle on the small configurations (cube, subdomain, adjoint copy) and exit")
    ap.add_argument("--cpu-omp-only", action="store_true",
                    help="time only the OpenMP build of the oracle on a crop and print its record")
    ap.add_argument("--cpu-crop", type=int, nargs=2, default=(160, 160))
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--nx", type=int, default=800)
    ap.add_argument("--ny", type=int, default=800)
    ap.add_argument("--nz", type=int, default=128)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU slab decomposition is a design, not a measured path)", file=sys.stderr)
        sys.exit(2)

    if args.oracle_configs:
        print(json.dumps({"oracle_configs": oracle_configs()}), flush=True)
        return

    if args.cpu_omp_only:
        from paper_2607_04516_amd import workloads
        w = workloads.urban_km("f32", nx=args.nx, ny=args.ny, nz=args.nz)
        print(json.dumps(cpu_baseline(w, args.cpu_seconds, tuple(args.cpu_crop))), flush=True)
        return

    import torch

    from paper_2607_04516_amd import binding, workloads
    binding.load()
    torch.cuda.set_device(0)

    if args.copy_calibration:
        a = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return

    if args.adjoint_only:
        print("[bench] adjoint workload", file=sys.stderr, flush=True)
        print(json.dumps({"adjoint": time_adjoint(args.adjoint_steps)}), flush=True)
        return

    # the copy ceiling first, on a fresh device heap
    copy_gbs = copy_bandwidth()
    print(f"[bench] device copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    print(f"[bench] building workload {args.nx}x{args.ny}x{args.nz}", file=sys.stderr, flush=True)
    w = workloads.urban_km("f32", nx=args.nx, ny=args.ny, nz=args.nz)
    res = time_forward(w, args.storage, args.steps, args.warmup)
    print(f"[bench] {args.storage}: {res['mlups']:.0f} MLUPS, kernel {res['kernel_ms']:.3f} ms, "
          f"{res['achieved_gbs']:.0f} GB/s", file=sys.stderr, flush=True)

    extra = {}
    if not args.no_extra:
        for s in ("f16s", "bf16s"):
            r = time_forward(w, s, args.steps, args.warmup)
            tb, _ = traffic_from_profiles(s, w.name)
            extra[s] = {"value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 4),
                        "kernel_ms": round(r["kernel_ms"], 4), "achieved_gbs": round(r["achieved_gbs"], 1),
                        "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                        "traffic": None if tb is None else round(tb / (r["kernel_ms"] * 1e-3) / 1e9, 1),
                        "vs_f32_mlups": round(r["mlups"] / res["mlups"], 3)}
            print(f"[bench] {s}: {r['mlups']:.0f} MLUPS, {r['achieved_gbs']:.0f} GB/s", file=sys.stderr,
                  flush=True)

    feats = None
    if not args.no_features:
        print("[bench] features", file=sys.stderr, flush=True)
        feats = time_features(w, min(args.steps, 100), args.warmup)
        print(f"[bench] features: {feats}", file=sys.stderr, flush=True)

    vox = None
    if not args.no_voxelize:
        print("[bench] voxelizer", file=sys.stderr, flush=True)
        vox = time_voxelize()
        print(f"[bench] voxelize: {vox}", file=sys.stderr, flush=True)

    shard = None
    if not args.no_shard:
        print("[bench] 8-slab decomposition", file=sys.stderr, flush=True)
        shard = time_shard(w, 8, min(args.steps, 40), args.warmup)
        print(f"[bench] shard: {shard}", file=sys.stderr, flush=True)

    traffic, _ = traffic_from_profiles(args.storage, w.name)

    adj = None
    if not args.no_adjoint:
        # In a child process of its own: after the large forward grids above,
        # the same kernels run up to 15% slower in this process (its device
        # memory is fragmented by the freed 800x800x128 arrays), which is not
        # what a program running only the adjoint workload sees.
        print("[bench] adjoint workload (child process)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        adj = adjoint_child(args.adjoint_steps)
        print(f"[bench] adjoint: {adj}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a crop", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w)
        print("[bench] timing the OpenMP build of the oracle on a larger crop", file=sys.stderr, flush=True)
        cpu["openmp"] = cpu_baseline_openmp()

    line = {
        "metric": METRIC,
        "value": round(res["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: urban buildings PAF 0.30, median 12, power-law inflow 30 deg "
                               f"on x-/y-, outflow x+/y+, wall ground, free-slip top, tau0 0.505, C 0.1",
                   "cells": w.cells, "fluid_cells": res["fluid_cells"], "storage": args.storage,
                   "layout": res["layout"]},
        "roofline": {"bound": "hbm", "achieved": round(res["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(res["achieved_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / (res["kernel_ms"] * 1e-3) / 1e9, 1),
                     "traffic_bytes_per_launch": traffic,
                     "traffic_bytes_per_launch_request_sizes": traffic_request_sizes(args.storage, w.name),
                     "kernel": "lbm::k_even / lbm::k_odd (alternating A-A launches, averaged)",
                     "kernel_ms": round(res["kernel_ms"], 4),
                     "bytes_per_launch": res["bytes_per_launch"],
                     "device_copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(res["achieved_gbs"] / copy_gbs, 4)},
        "cpu_baseline": cpu,
    }
    if extra:
        line["storage_forms"] = extra
    if feats:
        line["features"] = feats
    if shard:
        line["shard"] = shard
    if vox:
        line["voxelize"] = vox
    if adj:
        line["adjoint"] = adj
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
