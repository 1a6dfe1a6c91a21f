"""Seeded synthetic inputs for the urban-wind LBM workloads.

This module builds inputs only: solid masks, inflow profiles, initial velocity
profiles and probe positions.  It holds none of the lattice-Boltzmann
arithmetic, imports neither the HIP binding nor the oracle, and is the one
module both of them are fed from.

Face kinds are given by name ("periodic", "inflow", "outflow", "freeslip",
"wall") in the face order x-, x+, y-, y+, z-, z+; each consumer maps the names
to its own enumeration.

The paper's Haixinsha domain (Sec. 3: 4 km x 4.5 km at 5 m, 800 m high, about
1.16e8 cells, 3D-GloBFP footprints and lidar-driven boundaries) is not
available; the urban generator below stands in for its building data and the
power-law profiles stand in for its reconstructed boundary winds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FACE_NAMES = ("periodic", "inflow", "outflow", "freeslip", "wall")

FACES_CHANNEL = ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip")
FACES_TWO_INLETS = ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip")
# the paper's open domain (Sec. 2.3): equilibrium velocity on the four lateral
# faces and the top, no-slip ground
FACES_OPEN = ("inflow", "inflow", "inflow", "inflow", "wall", "inflow")


# --------------------------------------------------------------------------
# Building masks
# --------------------------------------------------------------------------
def cube_mask(nx, ny, nz, x0=16, size=(8, 8, 12)):
    """One solid block on the ground: x in [x0, x0+sx), centred in y, z in [0, sz)."""
    sx, sy, sz = size
    m = np.zeros((nz, ny, nx), np.uint8)
    y0 = (ny - sy) // 2
    m[0:sz, y0:y0 + sy, x0:x0 + sx] = 1
    return m


def urban_heights(nx, ny, paf, median, sigma, hmax, seed, footprint=(10, 40),
                  margin_x=32, margin_y=4):
    """Height map [ny, nx] of axis-aligned rectangular buildings.

    Buildings are drawn until the covered fraction of the placement region
    reaches ``paf``: footprint sides uniform in ``footprint`` (inclusive),
    position uniform in the placement region (clipped to it), height
    lognormal ``round(median * exp(sigma * N(0,1)))`` clipped to [1, hmax].
    Overlaps keep the taller building.  The placement region keeps
    ``margin_x`` cells clear of the x faces and ``margin_y`` of the y faces.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.zeros((ny, nx), np.int32)
    x_lo, x_hi = margin_x, nx - margin_x
    y_lo, y_hi = margin_y, ny - margin_y
    if x_hi - x_lo < 1 or y_hi - y_lo < 1:
        raise ValueError("placement region is empty")
    area = (x_hi - x_lo) * (y_hi - y_lo)
    region = h[y_lo:y_hi, x_lo:x_hi]
    guard = 0
    while np.count_nonzero(region) < paf * area:
        w = int(rng.integers(footprint[0], footprint[1] + 1))
        l = int(rng.integers(footprint[0], footprint[1] + 1))
        x0 = int(rng.integers(x_lo, x_hi))
        y0 = int(rng.integers(y_lo, y_hi))
        hb = int(np.clip(round(median * math.exp(sigma * rng.standard_normal())), 1, hmax))
        xs, xe = x0, min(x0 + w, x_hi)
        ys, ye = y0, min(y0 + l, y_hi)
        blk = h[ys:ye, xs:xe]
        np.maximum(blk, hb, out=blk)
        guard += 1
        if guard > 1_000_000:
            raise RuntimeError("building generator did not reach the plan-area fraction")
    return h


def heights_to_mask(h, nz):
    """Solid mask [nz, ny, nx] (1 = solid) from a height map: cell z is solid below the roof."""
    z = np.arange(nz, dtype=np.int32)[:, None, None]
    return (z < h[None, :, :]).astype(np.uint8)


def probe_cells(h, nz, count, seed, margin_x=32, margin_y=4):
    """Integer probe cells (x, y, z) above roof level: (x, y) uniform in the
    placement region, z uniform in [h(x, y) + 2, nz - 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx = h.shape
    out = []
    while len(out) < count:
        x = int(rng.integers(margin_x, nx - margin_x))
        y = int(rng.integers(margin_y, ny - margin_y))
        lo, hi = int(h[y, x]) + 2, nz - 3
        if lo > hi:
            continue
        z = int(rng.integers(lo, hi + 1))
        out.append((x, y, z))
    return np.asarray(out, np.int32)


# --------------------------------------------------------------------------
# Velocity profiles ([nz, 3], lattice units, heights z + 1/2 above the ground plane)
# --------------------------------------------------------------------------
def uniform_profile(nz, u):
    return np.tile(np.asarray(u, np.float64), (nz, 1))


def power_law_speeds(nz, u_ref, z_ref, alpha):
    z = np.arange(nz, dtype=np.float64) + 0.5
    return u_ref * (z / z_ref) ** alpha


def direction_profile(speeds, theta_deg):
    """Profile s(z) (cos theta, sin theta, 0)."""
    t = math.radians(theta_deg)
    s = np.asarray(speeds, np.float64)
    return np.stack([s * math.cos(t), s * math.sin(t), np.zeros_like(s)], axis=1)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    faces: tuple
    tau0: float
    c_smag: float
    storage: str
    steps: int
    solid: np.ndarray
    inflow: dict            # face index -> [nz, 3] profile
    u0: np.ndarray          # [nz, 3] initial velocity profile
    noise_amp: float = 1e-4
    noise_seed: int = 0
    delta: float = 1.0
    force: tuple = (0.0, 0.0, 0.0)
    probes: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    heights: np.ndarray | None = None
    omega: tuple = (0.0, 0.0, 0.0)   # Earth rotation vector in lattice units (grid frame)
    sponge: tuple = (0, 0.0)         # (width W, strength s_max) of the sponge / buffer nudging

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    @property
    def fluid_cells(self):
        return int(self.cells - int(np.count_nonzero(self.solid)))


def cube_flow(storage="f64", steps=100, nx=64, ny=48, nz=32):
    """Single 8x8x12 block at x = 16 on the ground, uniform inflow (0.05, 0, 0),
    zero-gradient outflow, free-slip top and sides, bounce-back ground."""
    prof = uniform_profile(nz, (0.05, 0.0, 0.0))
    return Workload("cube_64x48x32", nx, ny, nz, FACES_CHANNEL, 0.52, 0.1, storage, steps,
                    cube_mask(nx, ny, nz), {0: prof}, prof.copy(), noise_seed=1)


def urban_block(storage="f32", steps=2000, nx=512, ny=512, nz=128, hmax=100, seed=2,
                probe_seed=3, noise_seed=4, nprobes=32, footprint=(10, 40), margin_x=32,
                margin_y=4, median=20):
    """Urban block: PAF 0.35 buildings, median height 20 (sigma 0.5), power-law
    inflow 0.08 ((z+1/2)/100)^0.25 along +x, tau0 0.505, C 0.1."""
    h = urban_heights(nx, ny, 0.35, median, 0.5, hmax, seed, footprint, margin_x, margin_y)
    prof = direction_profile(power_law_speeds(nz, 0.08, 100.0, 0.25), 0.0)
    probes = probe_cells(h, nz, nprobes, probe_seed, margin_x, margin_y) if nprobes else \
        np.zeros((0, 3), np.int32)
    return Workload(f"urban_{nx}x{ny}x{nz}", nx, ny, nz, FACES_CHANNEL, 0.505, 0.1, storage,
                    steps, heights_to_mask(h, nz), {0: prof}, prof.copy(), noise_seed=noise_seed,
                    probes=probes, heights=h)


def urban_km(storage="f32", steps=5000, nx=800, ny=800, nz=128, seed=5, noise_seed=6):
    """Kilometre-scale analogue: PAF 0.30, median height 12, power-law inflow
    (alpha 0.22, 0.08 at z = 100) at 30 degrees on the x- and y- faces."""
    h = urban_heights(nx, ny, 0.30, 12, 0.5, 100, seed, (10, 40), 32, 32)
    prof = direction_profile(power_law_speeds(nz, 0.08, 100.0, 0.22), 30.0)
    return Workload(f"urban_km_{nx}x{ny}x{nz}", nx, ny, nz, FACES_TWO_INLETS, 0.505, 0.1,
                    storage, steps, heights_to_mask(h, nz), {0: prof, 2: prof.copy()},
                    prof.copy(), noise_seed=noise_seed, heights=h)


def urban_km_open(storage="f32", steps=5000, sponge=(16, 0.05)):
    """The kilometre grid with the paper's open boundaries (Sec. 2.3): the
    30-degree power-law profile as the boundary state of all four lateral
    faces and the top (equilibrium velocity faces), no-slip ground, and the
    relaxation layers (width, strength) next to those faces."""
    w = urban_km(storage, steps)
    w.name = "urban_km_open_800x800x128"
    w.faces = FACES_OPEN
    prof = w.inflow[0]
    w.inflow = {F: prof.copy() for F in (0, 1, 2, 3, 5)}
    w.sponge = sponge
    return w


def urban_subdomain(storage="f16s", steps=100):
    """128x128x64 copy of the urban block for oracle comparisons (heights clipped to 48)."""
    return urban_block(storage, steps, 128, 128, 64, hmax=48, nprobes=0)


def adjoint_urban(storage="f32", steps=1000, nx=256, ny=256, nz=96, small=False):
    """Adjoint workload: PAF 0.35, median 20, heights clipped to 80, 24 probes,
    inflow = per-height speeds along angle theta on the x- face.
    ``small`` gives the 64x64x32 copy with footprints, heights and margins scaled by 1/4."""
    if small:
        nx, ny, nz = 64, 64, 32
        w = urban_block(storage, steps, nx, ny, nz, hmax=20, seed=7, probe_seed=8, noise_seed=9,
                        nprobes=24, footprint=(3, 10), margin_x=8, margin_y=2, median=5)
    else:
        w = urban_block(storage, steps, nx, ny, nz, hmax=80, seed=7, probe_seed=8, noise_seed=9,
                        nprobes=24)
    w.name = f"adjoint_urban_{nx}x{ny}x{nz}"
    return w


def face_profiles(w: Workload) -> np.ndarray:
    """Inflow profiles of a workload as a dense [6, nz, 3] array (zeros where unused)."""
    out = np.zeros((6, w.nz, 3))
    for k, v in w.inflow.items():
        out[k] = v
    return out


# --------------------------------------------------------------------------
# Synthetic building meshes (closed triangle meshes in lattice units) for the
# voxelizer: the 3D building footprints of the paper's study area are not
# available, so boxes and rotated prisms stand in.
# --------------------------------------------------------------------------
_BOX_FACES = np.array([(0, 2, 1), (0, 3, 2), (4, 5, 6), (4, 6, 7), (0, 1, 5), (0, 5, 4), (1, 2, 6), (1, 6, 5),
                       (2, 3, 7), (2, 7, 6), (3, 0, 4), (3, 4, 7)])


def box_mesh(x0, x1, y0, y1, z0, z1):
    """[12, 3, 3] triangles of the box [x0, x1] x [y0, y1] x [z0, z1], outward."""
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], np.float64)
    return v[_BOX_FACES]


def prism_mesh(cx, cy, w, l, angle, z0, z1):
    """A w x l rectangle centred at (cx, cy), turned by `angle` (radians),
    extruded from z0 to z1: [12, 3, 3] triangles."""
    c, s = math.cos(angle), math.sin(angle)
    pts = []
    for dx, dy in ((-w / 2, -l / 2), (w / 2, -l / 2), (w / 2, l / 2), (-w / 2, l / 2)):
        pts.append((cx + c * dx - s * dy, cy + s * dx + c * dy))
    v = np.array([[p[0], p[1], z0] for p in pts] + [[p[0], p[1], z1] for p in pts], np.float64)
    return v[_BOX_FACES]


def octahedron_mesh(cx, cy, cz, r):
    """[8, 3, 3] triangles of |x - cx| + |y - cy| + |z - cz| = r."""
    P = [(cx + r, cy, cz), (cx - r, cy, cz), (cx, cy + r, cz), (cx, cy - r, cz), (cx, cy, cz + r), (cx, cy, cz - r)]
    faces = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    return np.array([[P[i] for i in f] for f in faces], np.float64)


def meshes_to_arrays(meshes):
    """(triangles [nt, 3, 3], mesh starts [nm + 1]) from a list of meshes."""
    starts = np.zeros(len(meshes) + 1, np.int32)
    for i, m in enumerate(meshes):
        starts[i + 1] = starts[i] + len(m)
    tris = np.concatenate(meshes).astype(np.float64) if meshes else np.zeros((0, 3, 3))
    return tris, starts


def urban_box_meshes(nx, ny, paf, median, sigma, hmax, seed, footprint=(10, 40), margin_x=32, margin_y=4):
    """The buildings of urban_heights as box meshes (the same draws), so their
    voxelization equals heights_to_mask(urban_heights(...))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.zeros((ny, nx), np.int32)
    x_lo, x_hi, y_lo, y_hi = margin_x, nx - margin_x, margin_y, ny - margin_y
    area = (x_hi - x_lo) * (y_hi - y_lo)
    region = h[y_lo:y_hi, x_lo:x_hi]
    meshes = []
    while np.count_nonzero(region) < paf * area:
        w = int(rng.integers(footprint[0], footprint[1] + 1))
        l = int(rng.integers(footprint[0], footprint[1] + 1))
        x0 = int(rng.integers(x_lo, x_hi))
        y0 = int(rng.integers(y_lo, y_hi))
        hb = int(np.clip(round(median * math.exp(sigma * rng.standard_normal())), 1, hmax))
        xs, xe = x0, min(x0 + w, x_hi)
        ys, ye = y0, min(y0 + l, y_hi)
        blk = h[ys:ye, xs:xe]
        np.maximum(blk, hb, out=blk)
        meshes.append(box_mesh(xs, xe, ys, ye, 0, hb))
    return meshes


def rotated_building_meshes(nx, ny, count, seed, footprint=(6.0, 30.0), hmax=60.0, margin=8.0):
    """Rotated rectangular prisms with lognormal heights: general triangles
    for the voxelizer (no axis-aligned faces)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        w, l = rng.uniform(*footprint, 2)
        cx = rng.uniform(margin + 20, nx - margin - 20)
        cy = rng.uniform(margin + 20, ny - margin - 20)
        hb = float(np.clip(12.0 * math.exp(0.5 * rng.standard_normal()), 2.0, hmax))
        out.append(prism_mesh(cx, cy, w, l, rng.uniform(0.0, math.pi), 0.0, hb))
    return out
