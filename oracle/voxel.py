"""Oracle of the ray-parity voxelizer (Sec. 4.1: the triangle mesh is
voxelized by casting axis-aligned rays through grid columns, intersecting
them with the triangles and applying the odd-even parity rule along each
column; independent passes along different ray directions corroborate the
solid labels; Sec. 2.1: the solid mask is the Boolean union of the layers).

TEST INFRASTRUCTURE ONLY: plain FP64 numpy; only tests/, the smoke check and
the benchmark's CPU baseline may use it.

Definitions (readings where the paper gives one sentence):
  * cell (x, y, z) has its centre at (x + 1/2, y + 1/2, z + 1/2) in lattice
    units; a pass along axis a casts one ray per column of the other two
    axes through the cell centres;
  * each closed mesh (a building) is tested on its own and the results are
    united, so overlapping buildings stay solid;
  * a ray crosses a triangle where its foot (u, v) lies inside the
    triangle's projection onto the (u, v) plane, (u, v) = (x, y) for rays
    along z, (y, z) along x, (z, x) along y; the projection is taken
    counter-clockwise and a foot on an edge counts for the triangle only if
    the edge runs upward (B_v > A_v) or is horizontal and runs in -u, so a
    shared edge counts once; triangles seen edge-on are skipped;
  * with edge functions E(P; A, B) = (B_u - A_u)(P_v - A_v) - (B_v - A_v)(P_u - A_u)
    and w0 = E(P; B, C), w1 = E(P; C, A), w2 = E(P; A, B), the crossing
    coordinate along the ray is t = (w0 A_t + w1 B_t + w2 C_t) / (w0 + w1 + w2);
  * a cell is inside a mesh when the number of crossings with t below its
    centre coordinate is odd;
  * one pass (z) labels directly; three passes (z, x, y) label a cell solid
    when at least two of them find it inside.
The results are OR-ed into the given mask.
"""
from __future__ import annotations

import numpy as np

# (u, v, t) axes of a pass along each ray axis
PASS_AXES = {2: (0, 1, 2), 0: (1, 2, 0), 1: (2, 0, 1)}


def edge(pu, pv, au, av, bu, bv):
    return (bu - au) * (pv - av) - (bv - av) * (pu - au)


def _counts(e, au, av, bu, bv):
    """Whether a foot with edge value e counts for edge A -> B (the tie rule)."""
    return (e > 0.0) | ((e == 0.0) & ((bv > av) | ((bv == av) & (bu < au))))


def pass_inside(shape, tris, starts, axis):
    """Inside mask [nz, ny, nx] (bool) of one pass along `axis` (0 x, 1 y, 2 z)."""
    nz, ny, nx = shape
    n = (nx, ny, nz)
    ua, va, ta = PASS_AXES[axis]
    nu, nv, nt = n[ua], n[va], n[ta]
    pu = (np.arange(nu) + 0.5)[:, None] * np.ones((1, nv))       # [nu, nv] ray feet
    pv = np.ones((nu, 1)) * (np.arange(nv) + 0.5)[None, :]
    centres = np.arange(nt) + 0.5
    out = np.zeros((nu, nv, nt), bool)
    tris = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    for m in range(len(starts) - 1):
        parity = np.zeros((nu, nv, nt), bool)
        for tri in tris[starts[m]:starts[m + 1]]:
            a, b, c = tri[0], tri[1], tri[2]
            area = edge(c[ua], c[va], a[ua], a[va], b[ua], b[va])
            if area == 0.0:
                continue                      # seen edge-on
            if area < 0.0:
                b, c = c, b                   # counter-clockwise in the projection
            w0 = edge(pu, pv, b[ua], b[va], c[ua], c[va])
            w1 = edge(pu, pv, c[ua], c[va], a[ua], a[va])
            w2 = edge(pu, pv, a[ua], a[va], b[ua], b[va])
            hit = (_counts(w0, b[ua], b[va], c[ua], c[va]) & _counts(w1, c[ua], c[va], a[ua], a[va])
                   & _counts(w2, a[ua], a[va], b[ua], b[va]))
            if not hit.any():
                continue
            t = (w0 * a[ta] + w1 * b[ta] + w2 * c[ta]) / (w0 + w1 + w2)
            # cells whose centre lies above the crossing flip
            parity ^= hit[:, :, None] & (centres[None, None, :] > t[:, :, None])
        out |= parity
    # (u, v, t) -> (x, y, z) -> [nz, ny, nx]
    xyz = np.moveaxis(out, (0, 1, 2), (ua, va, ta))
    return np.ascontiguousarray(np.transpose(xyz, (2, 1, 0)))


def voxelize(shape, tris, starts, passes=1, solid=None):
    """Solid mask [nz, ny, nx] uint8: the given mask OR the voxelized meshes."""
    out = np.zeros(shape, np.uint8) if solid is None else np.array(solid, np.uint8, copy=True)
    if passes == 1:
        lab = pass_inside(shape, tris, starts, 2)
    elif passes == 3:
        votes = sum(pass_inside(shape, tris, starts, a).astype(np.int32) for a in (2, 0, 1))
        lab = votes >= 2
    else:
        raise ValueError("passes must be 1 or 3")
    out |= lab.astype(np.uint8)
    return out
