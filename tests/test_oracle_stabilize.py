"""Pins of the oracle's open-boundary stabilisers: flux balancing and the
sponge / buffer nudging (Sec. 2.2 and 2.3)."""
import numpy as np
import pytest

import oracle
from oracle import FREESLIP, INFLOW_EQ, OUTFLOW_ZG, WALL
from oracle import stabilize as st


def _open_box(nx=10, ny=8, nz=6, seed=0):
    faces = [INFLOW_EQ, INFLOW_EQ, INFLOW_EQ, INFLOW_EQ, WALL, INFLOW_EQ]
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8)
    profiles = {f: rng.normal(0.0, 0.03, (nz, 3)) + np.array([0.05, 0.02, 0.0]) for f in (0, 1, 2, 3, 5)}
    return faces, solid, profiles


def _field(faces, solid, profiles):
    nz, ny, nx = solid.shape
    fld = np.zeros((nz, ny, nx, 3))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                f = st.owner(faces, nx, ny, nz, x, y, z)
                if f >= 0:
                    fld[z, y, x] = profiles[f][z]
    return fld


def test_two_face_channel_worked_example():
    """x- face 0.05 in, x+ face 0.04 out, walls elsewhere: the net flux is
    -0.01 per row pair, and the balanced faces both carry 0.045."""
    nx, ny, nz = 6, 5, 4
    faces = [INFLOW_EQ, INFLOW_EQ, FREESLIP, FREESLIP, WALL, WALL]
    solid = np.zeros((nz, ny, nx), np.uint8)
    prof = {0: np.tile([0.05, 0.0, 0.0], (nz, 1)), 1: np.tile([0.04, 0.0, 0.0], (nz, 1))}
    phi, n = st.net_flux_profiles(faces, solid, prof)
    assert n == 2 * ny * nz
    assert abs(phi - ny * nz * (-0.05 + 0.04)) <= 1e-15
    out, before, after = st.balance_profiles(faces, solid, prof)
    np.testing.assert_allclose(out[0][:, 0], 0.045, rtol=1e-14)
    np.testing.assert_allclose(out[1][:, 0], 0.045, rtol=1e-14)
    assert abs(after) <= 1e-15


def test_balance_is_the_minimum_norm_correction():
    faces, solid, profiles = _open_box()
    fld = _field(faces, solid, profiles)
    out, phi, after = st.balance_field(faces, solid, fld)
    c = st.boundary_cells(faces, solid)
    n_out = st.NORMALS_OUT[c[:, 0]]
    delta = np.einsum("na,na->n", (out - fld)[c[:, 3], c[:, 2], c[:, 1]], n_out)
    # least-squares minimum-norm solution of sum(delta) = -phi (library routine)
    ref = np.linalg.lstsq(np.ones((1, len(c))), np.array([-phi]), rcond=None)[0]
    np.testing.assert_allclose(delta, ref, atol=1e-16)
    # only the normal components moved
    tang = (out - fld)[c[:, 3], c[:, 2], c[:, 1]] - delta[:, None] * n_out
    assert np.abs(tang).max() <= 1e-17
    scale = np.abs(np.einsum("na,na->n", fld[c[:, 3], c[:, 2], c[:, 1]], n_out)).sum()
    assert abs(phi) > 1e-3 and abs(after) <= 1e-14 * scale
    # any other zero-flux correction is larger
    rng = np.random.default_rng(1)
    for _ in range(5):
        d = ref + rng.normal(0, 1e-3, len(c))
        d -= d.mean() - ref.mean()
        assert abs(d.sum() + phi) <= 1e-12 and np.linalg.norm(d) > np.linalg.norm(ref)


def test_profile_and_field_balancing_agree():
    faces, solid, profiles = _open_box(seed=3)
    out_p, phi_p, _ = st.balance_profiles(faces, solid, profiles)
    out_f, phi_f, _ = st.balance_field(faces, solid, _field(faces, solid, profiles))
    assert abs(phi_p - phi_f) <= 1e-15 * len(st.boundary_cells(faces, solid))
    fp = _field(faces, solid, out_p)
    c = st.boundary_cells(faces, solid)
    np.testing.assert_allclose(fp[c[:, 3], c[:, 2], c[:, 1]], out_f[c[:, 3], c[:, 2], c[:, 1]], atol=1e-16)


def test_sponge_strength_ramp_and_faces():
    faces = [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, FREESLIP, INFLOW_EQ, INFLOW_EQ]
    nx, ny, nz, W, s = 20, 18, 16, 4, 0.2
    for d in range(0, 7):
        got, f = st.sponge_strength(faces, nx, ny, nz, W, s, d, 9, 8)
        want = s * ((W + 1 - d) / W) ** 2 if 1 <= d <= W else 0.0
        assert abs(got - want) <= 1e-16 and (f == 0 if want else f == -1)
    # outflow, free-slip and the ground are never nudged
    assert st.sponge_strength(faces, nx, ny, nz, W, s, nx - 2, 9, 8)[0] == 0.0
    assert st.sponge_strength(faces, nx, ny, nz, W, s, 10, ny - 2, 8)[0] == 0.0
    assert st.sponge_strength(faces, nx, ny, nz, W, s, 10, 9, 1)[0] == 0.0
    # top sponge, and a corner takes the stronger layer
    assert st.sponge_strength(faces, nx, ny, nz, W, s, 10, 9, nz - 2) == (s, 5)
    got, f = st.sponge_strength(faces, nx, ny, nz, W, s, 2, 1, nz - 3)
    assert f == 2 and abs(got - s) <= 1e-16


def _sponge_oracle(W=3, s=0.25, c_smag=0.1):
    nx, ny, nz = 12, 10, 9
    faces = [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, FREESLIP, WALL, INFLOW_EQ]
    prof = np.tile([0.06, 0.015, 0.0], (nz, 1))
    prof[:, 0] *= np.linspace(0.5, 1.0, nz)
    inflow = {0: prof, 2: prof, 5: prof}
    o = oracle.Oracle(nx, ny, nz, faces, tau0=0.54, c_smag=c_smag, inflow=inflow, sponge=(W, s))
    return o, faces, inflow


@pytest.mark.parametrize("cell", [(1, 5, 4), (2, 5, 4), (3, 5, 4), (4, 5, 4), (6, 1, 4), (6, 5, 7), (1, 1, 7)])
def test_collide_cell_is_collision_plus_nudge(cell):
    o, faces, inflow = _sponge_oracle()
    x, y, z = cell
    rng = np.random.default_rng(x + 10 * y + 100 * z)
    f = oracle.equilibrium(1.01, [0.03, -0.01, 0.02]) * (1 + 0.02 * (rng.random(19) - 0.5))
    got = o.collide_cell(f, x, y, z)
    fstar, rho, u, _ = o.collide(f)
    s, face = st.sponge_strength(faces, o.shape[2], o.shape[1], o.shape[0], 3, 0.25, x, y, z)
    if face < 0:
        np.testing.assert_array_equal(got, fstar)
        return
    ut = st.target_velocity(inflow, face, o.shape[0], z)
    np.testing.assert_allclose(got, st.nudge(fstar, rho, u, ut, s), rtol=0, atol=1e-16)
    # mass unchanged, momentum relaxed by s rho (u_t - u)
    c, _, _ = oracle.lattice()
    assert abs(got.sum() - fstar.sum()) <= 1e-15
    np.testing.assert_allclose(c.T.astype(float) @ (got - fstar), s * rho * (ut - u), atol=1e-16)


def test_target_state_is_a_fixed_point_of_the_nudging():
    """A uniform flow at the faces' common target velocity: the sponge adds nothing."""
    nx, ny, nz = 10, 8, 7
    faces = [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, FREESLIP, FREESLIP, INFLOW_EQ]
    u = np.array([0.05, 0.0, 0.0])      # tangential to the free-slip faces
    inflow = {f: np.tile(u, (nz, 1)) for f in (0, 2, 5)}
    a = oracle.Oracle(nx, ny, nz, faces, tau0=0.54, c_smag=0.1, inflow=inflow, sponge=(3, 0.3))
    f0 = a.init(u0=u, amp=0.0)
    f = a.run(f0, 10)
    assert np.abs(f - f0).max() <= 1e-15


def test_sponge_damps_deviation_near_the_face():
    o, faces, inflow = _sponge_oracle(W=3, s=0.3)
    plain = oracle.Oracle(12, 10, 9, faces, tau0=0.54, c_smag=0.1, inflow=inflow)
    f0 = o.init(u0=[0.0, 0.0, 0.0], amp=1e-3, seed=2)
    fa, fb = o.run(f0, 15), plain.run(f0, 15)
    _, ua, _ = o.macros(fa)
    _, ub, _ = plain.macros(fb)
    tgt = inflow[5][-1]
    top = (slice(None), slice(o.shape[0] - 4, o.shape[0] - 1), slice(3, 8), slice(4, 9))
    da = np.abs(ua[top] - tgt[:, None, None, None]).mean()
    db = np.abs(ub[top] - tgt[:, None, None, None]).mean()
    assert da < 0.8 * db


def test_oracle_adjoint_refuses_sponge():
    o, faces, inflow = _sponge_oracle()
    f = o.init(u0=[0.05, 0.0, 0.0], amp=0.0)
    with pytest.raises(RuntimeError):
        o.adjoint_step(f, np.zeros_like(f))
