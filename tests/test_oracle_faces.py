"""Pins of the oracle's per-cell boundary states (the face-wise mapped
boundary field of Sec. 2.3, App. F's U_b,i): a per-cell array per face in
place of the per-height profile, read by the inflow cells, the sponge /
buffer targets, flux balancing and the synthetic-inflow generator."""
import numpy as np
import pytest

import oracle
from oracle import FREESLIP, INFLOW_EQ, OUTFLOW_ZG, WALL, face_shape
from oracle import stabilize as st
from oracle import vk

FACES = [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, FREESLIP, WALL, INFLOW_EQ]


def _face_arrays(nx, ny, nz, seed=0):
    """Random per-cell boundary states on the INFLOW_EQ faces x-, y-, z+."""
    rng = np.random.default_rng(seed)
    out = {}
    for f in (0, 2, 5):
        n2, n1 = face_shape(f, nx, ny, nz)
        out[f] = np.array([0.04, 0.01, 0.0]) + rng.normal(0.0, 0.01, (n2, n1, 3))
    return out


def _face_cell(f, x, y, z):
    """(j2, j1) of cell (x, y, z) in face f's array, written out per axis."""
    if f in (0, 1):
        return z, y
    if f in (2, 3):
        return z, x
    return y, x


def test_face_shapes():
    assert face_shape(0, 7, 5, 4) == (4, 5)
    assert face_shape(3, 7, 5, 4) == (4, 7)
    assert face_shape(5, 7, 5, 4) == (5, 7)


def test_broadcast_arrays_reproduce_the_profiles_exactly():
    """Face arrays that repeat each face's profile along the face give the
    same run, bit for bit, as the profiles themselves (sponge on)."""
    nx, ny, nz = 10, 8, 7
    rng = np.random.default_rng(1)
    solid = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    prof = {f: np.array([0.04, 0.01, 0.0]) + rng.normal(0.0, 0.01, (nz, 3)) for f in (0, 2, 5)}
    arrays = {}
    for f, p in prof.items():
        n2, n1 = face_shape(f, nx, ny, nz)
        if f == 5:
            arrays[f] = np.broadcast_to(p[nz - 1], (n2, n1, 3)).copy()
        else:
            arrays[f] = np.broadcast_to(p[:, None, :], (n2, n1, 3)).copy()
    kw = dict(tau0=0.54, c_smag=0.12, solid=solid, sponge=(2, 0.2))
    a = oracle.Oracle(nx, ny, nz, FACES, inflow=prof, **kw)
    b = oracle.Oracle(nx, ny, nz, FACES, inflow=arrays, **kw)
    f0 = a.init(u0=[0.03, 0.0, 0.0], amp=1e-3, seed=3)
    np.testing.assert_array_equal(a.run(f0, 4), b.run(f0, 4))


def test_inflow_cells_hold_the_equilibrium_of_their_own_cell():
    nx, ny, nz = 9, 7, 6
    arrays = _face_arrays(nx, ny, nz, seed=2)
    o = oracle.Oracle(nx, ny, nz, FACES, tau0=0.55, inflow=arrays)
    f1 = o.run(o.init(u0=[0.02, 0.0, 0.0], amp=1e-3, seed=1), 1)
    checked = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f = st.owner(FACES, nx, ny, nz, x, y, z)
                if f < 0:
                    continue
                want = oracle.equilibrium(1.0, arrays[f][_face_cell(f, x, y, z)])
                np.testing.assert_allclose(f1[:, z, y, x], want, rtol=0, atol=1e-16)
                checked += 1
    assert checked > 2 * ny * nz


@pytest.mark.parametrize("cell", [(1, 4, 3), (2, 5, 2), (4, 1, 3), (5, 3, 4), (6, 2, 5), (1, 1, 4)])
def test_sponge_target_is_the_state_at_the_projection(cell):
    nx, ny, nz = 10, 9, 7
    arrays = _face_arrays(nx, ny, nz, seed=4)
    W, s = 3, 0.25
    o = oracle.Oracle(nx, ny, nz, FACES, tau0=0.54, c_smag=0.1, inflow=arrays, sponge=(W, s))
    x, y, z = cell
    rng = np.random.default_rng(x + 10 * y + 100 * z)
    fc = oracle.equilibrium(1.01, [0.03, -0.01, 0.02]) * (1 + 0.02 * (rng.random(19) - 0.5))
    got = o.collide_cell(fc, x, y, z)
    fstar, rho, u, _ = o.collide(fc)
    strength, face = st.sponge_strength(FACES, nx, ny, nz, W, s, x, y, z)
    assert face >= 0
    # the projection of (x, y, z) onto the face, indexed by hand
    ut = arrays[face][_face_cell(face, x, y, z)]
    np.testing.assert_allclose(got, st.nudge(fstar, rho, u, ut, strength), rtol=0, atol=1e-16)
    np.testing.assert_array_equal(st.target_velocity(arrays, face, nz, z, x, y), ut)


def test_flux_balance_of_face_arrays():
    nx, ny, nz = 10, 8, 6
    faces = [INFLOW_EQ, INFLOW_EQ, INFLOW_EQ, INFLOW_EQ, WALL, INFLOW_EQ]
    rng = np.random.default_rng(6)
    solid = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8)
    arrays = {}
    for f in (0, 1, 2, 3, 5):
        n2, n1 = face_shape(f, nx, ny, nz)
        arrays[f] = np.array([0.05, 0.02, 0.0]) + rng.normal(0.0, 0.02, (n2, n1, 3))
    out, phi, after = st.balance_profiles(faces, solid, arrays)
    c = st.boundary_cells(faces, solid)
    assert abs(phi) > 1e-3 and abs(after) <= 1e-14 * len(c)
    # the same as balancing the per-cell field of the owned boundary cells
    fld = np.zeros((nz, ny, nx, 3))
    for f, x, y, z in c:
        fld[z, y, x] = arrays[f][_face_cell(f, x, y, z)]
    out_f, phi_f, _ = st.balance_field(faces, solid, fld)
    assert abs(phi - phi_f) <= 1e-15 * len(c)
    for f, x, y, z in c:
        np.testing.assert_allclose(out[f][_face_cell(f, x, y, z)], out_f[z, y, x], atol=1e-16)
    # every entry of a face moved by the same normal shift
    for f in arrays:
        d = (out[f] - arrays[f]).reshape(-1, 3)
        np.testing.assert_allclose(d, np.broadcast_to(-(phi / len(c)) * st.NORMALS_OUT[f], d.shape), atol=1e-17)


def test_turbulence_takes_the_per_cell_mean_velocity():
    nx, ny, nz = 12, 9, 8
    arrays = _face_arrays(nx, ny, nz, seed=8)
    solid = np.zeros((nz, ny, nx), np.uint8)
    p = vk.VKParams(n_modes=16, length_scale=4.0, intensity=0.2, seed=5)
    gen = vk.VonKarmanInflow(FACES, solid, arrays, p)
    for (f, x, y, z), ub in zip(gen.cells, gen.ub):
        np.testing.assert_array_equal(ub, arrays[f][_face_cell(f, x, y, z)])
    assert abs(gen.u_ref - np.mean(np.linalg.norm(gen.ub, axis=1))) <= 1e-15
    # U_i(t) - U_b,i = sigma_i q(x_i, t)
    t = 7
    fld = gen.field(t)
    q = gen.q(t)
    for k, (f, x, y, z) in enumerate(gen.cells):
        np.testing.assert_allclose(fld[z, y, x] - gen.ub[k], gen.sigma[k] * q[k], atol=1e-15)
