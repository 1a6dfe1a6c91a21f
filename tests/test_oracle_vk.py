"""Pins of the oracle's synthetic von Karman inflow (App. F) against the
paper's stated properties and closed forms of the spectrum."""
import math

import numpy as np
import pytest

import oracle
from oracle import FREESLIP, INFLOW_EQ, OUTFLOW_ZG, WALL
from oracle import vk


def _table(n=64, L=20.0, seed=3, r=0, gains=(1.0, 1.0, 1.0), u_ref=0.08, e_c=(1.0, 0.0, 0.0)):
    p = vk.VKParams(n_modes=n, length_scale=L, seed=seed, gains=gains)
    return vk.mode_table(p, r, u_ref, np.array(e_c))


def test_splitmix_uniforms_in_unit_interval():
    u = [vk.uniform(7, r, m, j) for r in range(3) for m in range(20) for j in range(6)]
    assert min(u) >= 0.0 and max(u) < 1.0 and len(set(u)) == len(u)


@pytest.mark.parametrize("L", [5.0, 20.0, 300.0])
def test_wavenumber_band_and_log_stratification(L):
    n = 50
    k, amp, om, phi, kmag = _table(n=n, L=L)
    kmin, kmax = 2 * math.pi / (10 * L), math.pi
    assert np.all(kmag >= kmin) and np.all(kmag <= kmax)
    # one mode in each of the N equal bins of ln k
    bins = np.floor((np.log(kmag) - math.log(kmin)) / (math.log(kmax) - math.log(kmin)) * n).astype(int)
    assert np.array_equal(bins, np.arange(n))
    np.testing.assert_allclose(np.linalg.norm(k, axis=1), kmag, rtol=1e-14)


def test_degenerate_band_resets_kmin():
    # 2 pi / (10 L) >= pi when L <= 0.2
    k, amp, om, phi, kmag = _table(n=30, L=0.1)
    assert kmag.min() >= 0.1 * math.pi and kmag.max() <= math.pi
    assert kmag.min() < 0.1 * math.pi * 1.2


def test_isotropic_directions():
    k, amp, om, phi, kmag = _table(n=20000, L=20.0)
    kh = k / kmag[:, None]
    assert np.abs(kh.mean(axis=0)).max() < 0.02
    np.testing.assert_allclose(kh.T @ kh / len(kh), np.eye(3) / 3, atol=0.01)
    # phases uniform on [0, 2 pi)
    assert phi.min() >= 0.0 and phi.max() < 2 * math.pi
    assert abs(phi.mean() - math.pi) < 0.05


def test_von_karman_peak_and_inertial_range():
    """W(k) = k^4/(1+(kL)^2)^(17/6) peaks at kL = sqrt(12/5) and falls as
    k^(-5/3) (Kolmogorov) for kL >> 1."""
    L = 40.0
    k, amp, om, phi, kmag = _table(n=4000, L=L)
    a2 = amp[:, 0] ** 2
    kp = kmag[np.argmax(a2)]
    assert abs(kp * L - math.sqrt(12 / 5)) < 0.01 * math.sqrt(12 / 5)
    hi = kmag * L > 60
    slope = np.polyfit(np.log(kmag[hi]), np.log(a2[hi]), 1)[0]
    assert abs(slope + 5 / 3) < 0.01


def test_unit_rms_per_component_and_gains():
    """Unit RMS of each component before the gains (App. F), RMS = gain after."""
    g = (1.0, 0.5, 2.0)
    k, amp, om, phi, kmag = _table(n=64, L=20.0, gains=g)
    t = np.arange(0, 200000, 7.0)
    q = np.stack([vk.q_series(k, amp, om, phi, [[3.0, 5.0, 11.0]], tt)[0] for tt in t[:4000]])
    rms = np.sqrt((q ** 2).mean(axis=0))
    np.testing.assert_allclose(rms, g, rtol=0.08)
    # spatial average over many points at one time, same statement
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 5000, (20000, 3))
    qs = vk.q_series(k, amp, om, phi, x, 0.0)
    np.testing.assert_allclose(np.sqrt((qs ** 2).mean(axis=0)), g, rtol=0.05)


def test_frozen_convection_along_mean_flow():
    """q(x + u_ref tau e_c, t + tau) = q(x, t): the pattern moves with the mean flow."""
    e = np.array([math.cos(0.5), math.sin(0.5), 0.0])
    u_ref = 0.07
    k, amp, om, phi, kmag = _table(n=48, L=15.0, u_ref=u_ref, e_c=e)
    np.testing.assert_allclose(om, u_ref * (k @ e), rtol=1e-15)
    x = np.array([[4.0, 9.0, 2.0], [31.0, 0.0, 17.0]])
    for t, tau in [(0.0, 10.0), (123.0, 250.0)]:
        a = vk.q_series(k, amp, om, phi, x, t)
        b = vk.q_series(k, amp, om, phi, x + u_ref * tau * e, t + tau)
        np.testing.assert_allclose(b, a, atol=1e-10)
        c = vk.q_series(k, amp, om, phi, x - u_ref * tau * e, t + tau)
        assert np.abs(c - a).max() > 1e-3     # upstream is not the same pattern


def _channel(nx=9, ny=7, nz=6, faces=None, solid=None, prof=None):
    faces = faces or [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, FREESLIP, WALL, INFLOW_EQ]
    solid = np.zeros((nz, ny, nx), np.uint8) if solid is None else solid
    prof = np.tile([0.05, 0.02, 0.0], (nz, 1)) if prof is None else prof
    return faces, solid, {k: prof for k in range(6) if faces[k] == INFLOW_EQ}


def test_active_set_brute_force():
    nx, ny, nz = 9, 7, 6
    faces = [INFLOW_EQ, INFLOW_EQ, INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, INFLOW_EQ]
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0:2, 0, 4] = 1          # a solid cell on the y- face
    prof = np.tile([0.05, 0.02, 0.0], (nz, 1))
    profiles = {k: prof for k in range(6) if faces[k] == INFLOW_EQ}
    p = vk.VKParams()
    cells, ub, u_ref, e_c = vk.active_cells(faces, solid, profiles, p)
    want = set()
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid[z, y, x]:
                    continue
                on = [x == 0, x == nx - 1, y == 0, y == ny - 1, z == 0, z == nz - 1]
                fs = [k for k in range(6) if on[k] and faces[k] == INFLOW_EQ]
                if fs and fs[0] != 4:
                    want.add((fs[0], x, y, z))
    got = set(map(tuple, cells.tolist()))
    assert got == want
    assert len(got) == len(cells)              # each cell once
    assert not any(c[0] == 4 for c in got)     # bottom face excluded
    np.testing.assert_allclose(u_ref, np.linalg.norm([0.05, 0.02, 0.0]), rtol=1e-15)
    np.testing.assert_allclose(e_c, np.array([0.05, 0.02, 0.0]) / np.linalg.norm([0.05, 0.02, 0.0]), rtol=1e-14)


def test_inflow_only_filter_and_face_discard():
    # the x+ face is INFLOW_EQ but its mean velocity leaves the domain
    nx, ny, nz = 8, 6, 5
    faces = [INFLOW_EQ, INFLOW_EQ, FREESLIP, FREESLIP, WALL, FREESLIP]
    prof = np.tile([0.05, 0.0, 0.0], (nz, 1))
    profiles = {0: prof, 1: prof}
    solid = np.zeros((nz, ny, nx), np.uint8)
    cells, *_ = vk.active_cells(faces, solid, profiles, vk.VKParams(inflow_only=True))
    assert set(cells[:, 0].tolist()) == {0}
    cells, *_ = vk.active_cells(faces, solid, profiles, vk.VKParams(inflow_only=False))
    assert set(cells[:, 0].tolist()) == {0, 1}
    # a face at rest is discarded (characteristic speed <= 1e-7)
    profiles = {0: prof, 1: np.zeros((nz, 3))}
    cells, *_ = vk.active_cells(faces, solid, profiles, vk.VKParams())
    assert set(cells[:, 0].tolist()) == {0}
    # normal-speed variant: a face with purely tangential flow is discarded
    profiles = {0: prof, 1: np.tile([0.0, 0.05, 0.0], (nz, 1))}
    cells, *_ = vk.active_cells(faces, solid, profiles, vk.VKParams(char_normal=True))
    assert set(cells[:, 0].tolist()) == {0}


def test_sigma_and_superposition():
    faces, solid, profiles = _channel()
    for I, s0 in [(0.15, 0.0), (0.0, 0.004)]:
        v = vk.VonKarmanInflow(faces, solid, profiles, vk.VKParams(intensity=I, sigma0=s0, seed=5))
        want = I * np.linalg.norm([0.05, 0.02, 0.0]) if I > 0 else s0
        np.testing.assert_allclose(v.sigma, want, rtol=1e-15)
        fld = v.field(3)
        c = v.cells
        got = fld[c[:, 3], c[:, 2], c[:, 1]]
        np.testing.assert_allclose(got - v.ub, v.sigma[:, None] * v.q(3.0), atol=1e-15)
    # cells on no inflow face are not part of the field
    assert np.all(fld[1:-1, 1:-1, 1:-1] == 0.0)


def test_global_coordinates_make_subdomains_consistent():
    """Two grids that tile one domain (origin offsets) give the same field on
    the shared face as the whole grid (App. F: phases from global coordinates)."""
    nx, ny, nz = 12, 6, 5
    faces = [INFLOW_EQ, OUTFLOW_ZG, FREESLIP, FREESLIP, WALL, FREESLIP]
    prof = np.tile([0.06, 0.01, 0.0], (nz, 1))
    whole = vk.VonKarmanInflow(faces, np.zeros((nz, ny, nx), np.uint8), {0: prof}, vk.VKParams(seed=9))
    fw = whole.field(17)
    # split in y: two subdomains of 3 rows each, with their own y origin
    parts = []
    for y0 in (0, 3):
        v = vk.VonKarmanInflow(faces, np.zeros((nz, 3, nx), np.uint8), {0: prof},
                               vk.VKParams(seed=9, origin=(0, y0, 0)))
        parts.append(v.field(17))
    np.testing.assert_allclose(np.concatenate(parts, axis=1)[:, :, 0], fw[:, :, 0], atol=1e-15)


def test_stride_hold_and_interpolation():
    faces, solid, profiles = _channel()
    hold = vk.VonKarmanInflow(faces, solid, profiles, vk.VKParams(seed=2, stride=4))
    lin = vk.VonKarmanInflow(faces, solid, profiles, vk.VKParams(seed=2, stride=4, interpolate=True))
    for t in (8, 9, 10, 11):
        np.testing.assert_allclose(hold.q_strided(t), hold.q(8.0), atol=1e-15)
    np.testing.assert_allclose(lin.q_strided(8), lin.q(8.0), atol=1e-15)
    np.testing.assert_allclose(lin.q_strided(10), 0.5 * (lin.q(8.0) + lin.q(12.0)), atol=1e-15)
    np.testing.assert_allclose(lin.q_strided(11), 0.25 * lin.q(8.0) + 0.75 * lin.q(12.0), atol=1e-15)


def test_oracle_step_takes_the_field():
    """A field equal to the profiles reproduces the profile run bit for bit;
    a perturbed field changes only what the inflow cells feed."""
    nx, ny, nz = 9, 7, 6
    faces, solid, profiles = _channel(nx, ny, nz)
    o = oracle.Oracle(nx, ny, nz, faces, tau0=0.55, c_smag=0.1, solid=solid, inflow=profiles)
    f0 = o.init(u0=[0.05, 0.02, 0.0], amp=1e-3, seed=1)
    ref = o.step(f0)
    v = vk.VonKarmanInflow(faces, solid, profiles, vk.VKParams(intensity=0.0, sigma0=0.0))
    o.inflow_field = v.field(0)
    assert np.array_equal(o.step(f0), ref)
    v = vk.VonKarmanInflow(faces, solid, profiles, vk.VKParams(intensity=0.2, seed=4))
    o.inflow_field = v.field(0)
    f1 = o.step(f0)
    assert np.abs(f1 - ref).max() > 1e-5
    # inflow cells hold feq(rho0, U_i)
    c = v.cells[0]
    u = o.inflow_field[c[3], c[2], c[1]]
    np.testing.assert_allclose(f1[:, c[3], c[2], c[1]], oracle.equilibrium(1.0, u), rtol=1e-15)
