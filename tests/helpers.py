"""Shared test helpers: build matching oracle and GPU lattices from one workload."""
import numpy as np

import oracle
from paper_2607_04516_amd import workloads

FACE_NUM = {"periodic": oracle.PERIODIC, "inflow": oracle.INFLOW_EQ, "outflow": oracle.OUTFLOW_ZG,
            "freeslip": oracle.FREESLIP, "wall": oracle.WALL}


def oracle_for(w: workloads.Workload):
    faces = [FACE_NUM[f] if isinstance(f, str) else int(f) for f in w.faces]
    o = oracle.Oracle(w.nx, w.ny, w.nz, faces, tau0=w.tau0, c_smag=w.c_smag, delta=w.delta,
                      force=w.force, solid=w.solid, inflow=w.inflow, omega=w.omega, sponge=w.sponge)
    return o


def oracle_init(o, w):
    return o.init(u0=w.u0, amp=w.noise_amp, seed=w.noise_seed)


def small_workload(nx, ny, nz, faces, solid=None, tau0=0.52, c_smag=0.1, u=(0.04, 0.01, 0.0),
                   storage="f64", force=(0.0, 0.0, 0.0), noise=1e-3, seed=5, inflow_faces=None,
                   omega=(0.0, 0.0, 0.0)):
    """Tiny workload with uniform velocity on every inflow face."""
    solid = np.zeros((nz, ny, nx), np.uint8) if solid is None else solid
    prof = workloads.uniform_profile(nz, u)
    fn = [f if isinstance(f, str) else {v: k for k, v in FACE_NUM.items()}[f] for f in faces]
    inflow = {k: prof.copy() for k, f in enumerate(fn) if f == "inflow"}
    return workloads.Workload(f"small_{nx}x{ny}x{nz}", nx, ny, nz, tuple(fn), tau0, c_smag, storage, 10,
                              solid, inflow, prof.copy(), noise_amp=noise, noise_seed=seed, force=force,
                              omega=tuple(omega))


def fluid_mask(w):
    """Boolean [nz, ny, nx]: non-solid cells that are not inflow cells."""
    m = ~w.solid.astype(bool)
    nx, ny, nz = w.nx, w.ny, w.nz
    for k, f in enumerate(w.faces):
        if f != "inflow":
            continue
        a, side = k // 2, k % 2
        idx = [slice(None)] * 3
        n = (nx, ny, nz)[a]
        idx[2 - a] = n - 1 if side else 0
        m[tuple(idx)] = False
    return m


# Face sets of the boundary matrix: every face kind on every axis, corners
# between inflow and outflow faces, two inflow faces, periodic wraps.
FACE_SETS = [
    ("periodic",) * 6,
    ("wall", "wall", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
    ("outflow", "inflow", "outflow", "outflow", "freeslip", "outflow"),
    ("periodic", "periodic", "wall", "wall", "inflow", "outflow"),
    ("freeslip", "freeslip", "periodic", "periodic", "freeslip", "freeslip"),
    ("outflow", "outflow", "outflow", "outflow", "outflow", "outflow"),
]


def window_index(pts, faces, nx, ny, nz):
    """Index arrays (zi, yi, xi), broadcastable to [n, 5, 5, 5], of the 5x5x5
    windows centred on the cells pts [n, 3] (x, y, z): coordinates wrap on
    an axis whose faces are periodic and are clamped otherwise (a pull never
    reaches past a non-periodic face, so clamped entries are never read)."""
    pts = np.asarray(pts, np.int64)
    d = np.arange(-2, 3)
    out = []
    for a, n in enumerate((nx, ny, nz)):
        v = pts[:, a, None] + d
        periodic = faces[2 * a] in ("periodic", oracle.PERIODIC)
        out.append(np.mod(v, n) if periodic else np.clip(v, 0, n - 1))
    xi, yi, zi = out
    return zi[:, :, None, None], yi[:, None, :, None], xi[:, None, None, :]


def windows_np(f, pts, faces, nx, ny, nz):
    """Windows [n, 19, 5, 5, 5] of a state f [19, nz, ny, nx]."""
    zi, yi, xi = window_index(pts, faces, nx, ny, nz)
    return np.ascontiguousarray(np.moveaxis(f[:, zi, yi, xi], 0, 1))
