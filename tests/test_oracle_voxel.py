"""Pins of the oracle's ray-parity voxelizer (Sec. 4.1 re-voxelization,
Sec. 2.1 Boolean union): closed-form solids, an independent ray-triangle
formula, ties on edges and vertices, and the corroboration of passes."""
import math

import numpy as np
import pytest

from oracle import voxel
from paper_2607_04516_amd import workloads as W

SHAPE = (20, 22, 24)   # nz, ny, nx


def _centres(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    return x, y, z


@pytest.mark.parametrize("passes", [1, 3])
def test_box_is_the_cells_with_centres_inside(passes):
    t, s = W.meshes_to_arrays([W.box_mesh(3, 11, 4, 17, 0, 9)])
    got = voxel.voxelize(SHAPE, t, s, passes)
    x, y, z = _centres(SHAPE)
    want = (x > 3) & (x < 11) & (y > 4) & (y < 17) & (z < 9)
    np.testing.assert_array_equal(got, want.astype(np.uint8))


@pytest.mark.parametrize("passes", [1, 3])
def test_octahedron_closed_form(passes):
    cx, cy, cz, r = 11.3, 10.7, 9.2, 6.13
    t, s = W.meshes_to_arrays([W.octahedron_mesh(cx, cy, cz, r)])
    got = voxel.voxelize(SHAPE, t, s, passes)
    x, y, z = _centres(SHAPE)
    d = np.abs(x - cx) + np.abs(y - cy) + np.abs(z - cz)
    assert np.abs(d - r).min() > 1e-6          # no centre on the surface
    np.testing.assert_array_equal(got, (d < r).astype(np.uint8))


@pytest.mark.parametrize("angle", [0.3, 1.1, 2.6])
def test_rotated_prism_half_spaces(angle):
    cx, cy, w, l, h = 12.1, 10.9, 11.0, 6.0, 13.7
    t, s = W.meshes_to_arrays([W.prism_mesh(cx, cy, w, l, angle, 0.0, h)])
    got = voxel.voxelize(SHAPE, t, s, 3)
    x, y, z = _centres(SHAPE)
    c, sn = math.cos(angle), math.sin(angle)
    u = c * (x - cx) + sn * (y - cy)          # coordinates in the prism's frame
    v = -sn * (x - cx) + c * (y - cy)
    want = (np.abs(u) < w / 2) & (np.abs(v) < l / 2) & (z < h)
    margin = np.minimum(np.minimum(np.abs(np.abs(u) - w / 2), np.abs(np.abs(v) - l / 2)), np.abs(z - h))
    ok = margin > 1e-9
    np.testing.assert_array_equal(got[ok], want[ok].astype(np.uint8))


def test_overlapping_buildings_unite_and_a_cavity_stays_empty():
    a = W.box_mesh(2, 12, 2, 12, 0, 10)
    b = W.box_mesh(8, 20, 6, 18, 0, 14)            # overlaps a
    outer = W.box_mesh(1, 23, 1, 21, 12, 19)
    inner = W.box_mesh(5, 9, 5, 9, 14, 17)[:, ::-1]  # reversed orientation: a cavity in the same mesh
    t, s = W.meshes_to_arrays([a, b, np.concatenate([outer, inner])])
    got = voxel.voxelize(SHAPE, t, s, 3)
    x, y, z = _centres(SHAPE)
    ina = (x > 2) & (x < 12) & (y > 2) & (y < 12) & (z < 10)
    inb = (x > 8) & (x < 20) & (y > 6) & (y < 18) & (z < 14)
    shell = ((x > 1) & (x < 23) & (y > 1) & (y < 21) & (z > 12) & (z < 19)
             & ~((x > 5) & (x < 9) & (y > 5) & (y < 9) & (z > 14) & (z < 17)))
    np.testing.assert_array_equal(got, (ina | inb | shell).astype(np.uint8))


def _moller_trumbore_inside(tris, p, d):
    """Parity of crossings of the ray p + s d (s > 0) with a closed mesh,
    by the Moller-Trumbore ray-triangle test (a different formula)."""
    n = 0
    for a, b, c in tris:
        e1, e2 = b - a, c - a
        h = np.cross(d, e2)
        det = e1 @ h
        if abs(det) < 1e-14:
            continue
        f = 1.0 / det
        q = p - a
        uu = f * (q @ h)
        if uu < 0 or uu > 1:
            continue
        qq = np.cross(q, e1)
        vv = f * (d @ qq)
        if vv < 0 or uu + vv > 1:
            continue
        if f * (e2 @ qq) > 0:
            n += 1
    return n % 2 == 1


def test_random_tetrahedra_against_an_independent_ray_test():
    rng = np.random.default_rng(3)
    shape = (10, 11, 12)
    for trial in range(4):
        v = rng.uniform(0.7, 9.3, (4, 3)) * np.array([1.2, 1.1, 1.0])
        tris = np.array([[v[0], v[1], v[2]], [v[0], v[1], v[3]], [v[0], v[2], v[3]], [v[1], v[2], v[3]]])
        t, s = W.meshes_to_arrays([tris])
        got = voxel.voxelize(shape, t, s, 1)
        # the ray from each centre toward -z: cells are inside iff the upward
        # ray from below crosses an odd number of times before the centre,
        # i.e. the downward ray from the centre does
        nz, ny, nx = shape
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    p = np.array([x + 0.5, y + 0.5, z + 0.5])
                    want = _moller_trumbore_inside(tris, p, np.array([0.0, 0.0, -1.0]))
                    assert bool(got[z, y, x]) == want, (trial, x, y, z)


def test_feet_on_edges_and_vertices_count_once():
    """A box with half-integer corners: the rays through the face boundary
    and through the split diagonal of the top and bottom faces still see an
    even number of crossings, cells strictly inside are solid and nothing
    above or below the box is."""
    t, s = W.meshes_to_arrays([W.box_mesh(3.5, 10.5, 4.5, 12.5, 2.5, 9.5)])
    x, y, z = _centres(SHAPE)
    for passes in (1, 3):
        got = voxel.voxelize(SHAPE, t, s, passes).astype(bool)
        strict_in = (x > 3.5) & (x < 10.5) & (y > 4.5) & (y < 12.5) & (z > 2.5) & (z < 9.5)
        outside = (x < 3.5) | (x > 10.5) | (y < 4.5) | (y > 12.5) | (z < 2.5) | (z > 9.5)
        assert got[strict_in].all() and not got[outside].any()
    # a diagonal through cell centres: the ray on the shared edge of the two top triangles
    d = np.array([[2.5, 2.5, 1.0], [8.5, 8.5, 1.0], [2.5, 8.5, 1.0]])
    tri2 = np.array([[2.5, 2.5, 1.0], [8.5, 2.5, 1.0], [8.5, 8.5, 1.0]])
    top = np.stack([d, tri2])
    bottom = top.copy()
    bottom[:, :, 2] = 6.0
    t, s = W.meshes_to_arrays([np.concatenate([top, bottom])])
    got = voxel.pass_inside((8, 10, 10), t, s, 2)
    # the slab between the two squares: every column strictly inside, and
    # the columns on the diagonal (x = y) too, each exactly once
    for k in range(3, 8):
        assert got[2, k, k] and got[5, k, k]
        assert not got[0, k, k] and not got[7, k, k]


def test_corroboration_repairs_a_leaking_mesh():
    """A box with one bottom triangle missing: the upward rays through the
    hole see one crossing, so the z pass alone labels the column above the
    roof; with three passes the other two outvote it."""
    tris = W.box_mesh(4, 14, 5, 15, 2, 12)
    leak = tris[1:]                                 # drop a bottom triangle
    t, s = W.meshes_to_arrays([leak])
    x, y, z = _centres(SHAPE)
    want = (x > 4) & (x < 14) & (y > 5) & (y < 15) & (z > 2) & (z < 12)
    one = voxel.voxelize(SHAPE, t, s, 1).astype(bool)
    three = voxel.voxelize(SHAPE, t, s, 3).astype(bool)
    assert (one != want).sum() > 20
    np.testing.assert_array_equal(three, want)


def test_ors_into_the_given_mask():
    base = np.zeros(SHAPE, np.uint8)
    base[0] = 1                                     # a base layer
    t, s = W.meshes_to_arrays([W.box_mesh(3, 6, 3, 6, 0, 4)])
    got = voxel.voxelize(SHAPE, t, s, 1, solid=base)
    assert got[0].all() and got[1:4, 3:6, 3:6].all() and got.sum() == SHAPE[1] * SHAPE[2] + 27
