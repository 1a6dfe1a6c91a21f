"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: lattice
isotropy (App. D), exact moment identities of the Hermite equilibrium, the
defining relation of the closed-form tau_eff (App. D), closed-form flows
(Poiseuille, Taylor-Green decay), conservation laws, the published splitmix64
outputs, and permutation / time-reversal properties of the streaming with
its boundary rules.  None of these needs the GPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import FREESLIP, INFLOW_EQ, OUTFLOW_ZG, PERIODIC, WALL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- lattice
def test_lattice_isotropy():
    c, w, opp = oracle.lattice()
    c = c.astype(np.float64)
    d = np.eye(3)
    assert len({tuple(v) for v in c.tolist()}) == 19
    assert all(np.abs(v).sum() <= 2 for v in c)          # rest, faces, edges only
    assert abs(w.sum() - 1.0) < 1e-16
    assert np.abs(np.einsum("i,ia->a", w, c)).max() < 1e-17
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3.0, atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-17
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)
    np.testing.assert_array_equal(c[opp], -c)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 0.9 + 0.2 * rng.random()
    u = 0.1 * (rng.random(3) - 0.5)
    c, w, _ = oracle.lattice()
    c = c.astype(np.float64)
    feq = oracle.equilibrium(rho, u)
    assert abs(feq.sum() - rho) <= 1e-15 * rho
    np.testing.assert_allclose(c.T @ feq, rho * u, atol=1e-16)
    np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, feq),
                               rho * (np.eye(3) / 3.0 + np.outer(u, u)), atol=2e-16)
    # the rest state is the weights times rho
    np.testing.assert_allclose(oracle.equilibrium(rho, [0, 0, 0]), rho * w, rtol=1e-16)


# ---------------------------------------------------------------- closure
@pytest.mark.parametrize("q,rho", [(0.0, 1.0), (1e-4, 1.0), (3e-3, 0.97), (0.5, 1.1)])
def test_tau_eff_root(q, rho):
    tau0, cs, delta = 0.505, 0.1, 1.0
    t = oracle.tau_eff(tau0, cs, delta, q, rho)
    # positive root of tau^2 - tau0 tau - (C Delta)^2 Q / (2 rho cs^4) = 0
    k = (cs * delta) ** 2 * q / (2.0 * rho * (1.0 / 3.0) ** 2)
    assert t > 0
    assert abs(t * t - tau0 * t - k) <= 1e-15 * max(1.0, t * t)
    # nu_eff = nu_0 + nu_t with nu_t = (C Delta)^2 |S| and |S| = Q / (2 rho cs^2 tau_eff)
    nu_eff = (t - 0.5) / 3.0
    nu0 = (tau0 - 0.5) / 3.0
    s = q / (2.0 * rho / 3.0 * t)
    assert abs(nu_eff - (nu0 + (cs * delta) ** 2 * s)) <= 1e-15
    assert oracle.tau_eff(tau0, 0.0, delta, q, rho) == tau0


@pytest.mark.parametrize("force", [(0, 0, 0), (1e-4, -2e-5, 3e-5)])
def test_collision_conserves(force):
    rng = np.random.default_rng(11)
    o = oracle.Oracle(3, 3, 3, [PERIODIC] * 6, tau0=0.53, c_smag=0.1, force=force)
    c, w, _ = oracle.lattice()
    f = oracle.equilibrium(1.02, [0.03, -0.01, 0.02]) * (1 + 0.05 * (rng.random(19) - 0.5))
    fs, rho, u, tau = o.collide(f)
    assert tau > 0.53
    assert abs(fs.sum() - f.sum()) < 1e-15
    # Guo forcing adds exactly F to the momentum of a cell per step
    np.testing.assert_allclose(c.T @ fs, c.T @ f + np.asarray(force), atol=2e-17)
    # Pi is the literal non-equilibrium second moment
    q, pi = o.q_invariant(f, oracle.equilibrium(rho, u))
    cf = c.astype(np.float64)
    pi_ref = np.einsum("ia,ib,i->ab", cf, cf, f - oracle.equilibrium(rho, u))
    np.testing.assert_allclose(pi, pi_ref, atol=1e-17)
    assert abs(q - math.sqrt(2.0 * (pi_ref ** 2).sum())) < 1e-16


def test_collision_tau_one_gives_equilibrium():
    o = oracle.Oracle(3, 3, 3, [PERIODIC] * 6, tau0=1.0, c_smag=0.0)
    f = oracle.equilibrium(1.0, [0.02, 0.0, 0.01])
    f = f + 1e-3 * np.sin(np.arange(19))
    fs, rho, u, tau = o.collide(f)
    np.testing.assert_allclose(fs, oracle.equilibrium(rho, u), atol=1e-17)


# ---------------------------------------------------------------- noise
def test_splitmix64_published_vectors():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    gamma = 0x9E3779B97F4A7C15
    for k, v in enumerate(vals):
        assert oracle.splitmix64((k * gamma) & (2 ** 64 - 1)) == v


def test_initial_noise_bounds_and_seed():
    o = oracle.Oracle(8, 6, 5, [PERIODIC] * 6, tau0=0.6)
    f1 = o.init(u0=[0.05, 0, 0], amp=1e-4, seed=7)
    f2 = o.init(u0=[0.05, 0, 0], amp=1e-4, seed=7)
    f3 = o.init(u0=[0.05, 0, 0], amp=1e-4, seed=8)
    assert np.array_equal(f1, f2) and not np.array_equal(f1, f3)
    rho, u, _ = o.macros(f1)
    np.testing.assert_allclose(rho, 1.0, atol=1e-15)
    assert np.abs(u[0] - 0.05).max() <= 1e-4 and np.abs(u[1:]).max() <= 1e-4
    assert np.abs(u[0] - 0.05).max() > 5e-5     # the noise is there


# ---------------------------------------------------------------- invariants
def _box(nx=10, ny=8, nz=7):
    s = np.zeros((nz, ny, nx), np.uint8)
    s[0:3, 2:5, 3:6] = 1
    s[4, 6, 1] = 1
    return s


@pytest.mark.parametrize("faces", [
    [WALL, WALL, FREESLIP, FREESLIP, WALL, FREESLIP],
    [PERIODIC, PERIODIC, WALL, WALL, FREESLIP, FREESLIP],
    [INFLOW_EQ, OUTFLOW_ZG, FREESLIP, FREESLIP, WALL, FREESLIP],
    [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, OUTFLOW_ZG, WALL, FREESLIP],
    [OUTFLOW_ZG, OUTFLOW_ZG, OUTFLOW_ZG, OUTFLOW_ZG, WALL, OUTFLOW_ZG],
])
def test_rest_state_invariance(faces):
    o = oracle.Oracle(10, 8, 7, faces, tau0=0.505, c_smag=0.1, solid=_box())
    f0 = o.init(u0=[0, 0, 0], amp=0.0)
    f = o.run(f0, 20)
    assert np.abs(f - f0).max() <= 1e-15


@pytest.mark.parametrize("faces", [
    [WALL, WALL, FREESLIP, FREESLIP, WALL, FREESLIP],
    [PERIODIC, PERIODIC, WALL, WALL, FREESLIP, FREESLIP],
    [PERIODIC, PERIODIC, PERIODIC, PERIODIC, WALL, WALL],
])
def test_mass_conservation_closed_box(faces):
    o = oracle.Oracle(10, 8, 7, faces, tau0=0.52, c_smag=0.1, solid=_box())
    f0 = o.init(u0=[0.02, -0.01, 0.0], amp=0.02, seed=3)
    m0, _ = o.mass(f0)
    f = o.run(f0, 50)
    m1, _ = o.mass(f)
    assert abs(m1 - m0) <= 1e-13 * m0


def test_momentum_conservation_periodic():
    c, _, _ = oracle.lattice()
    o = oracle.Oracle(9, 8, 7, [PERIODIC] * 6, tau0=0.52, c_smag=0.1)
    f0 = o.init(u0=[0.03, -0.02, 0.01], amp=0.02, seed=5)
    p0 = np.einsum("ia,izyx->a", c.astype(float), f0)
    f = o.run(f0, 40)
    p1 = np.einsum("ia,izyx->a", c.astype(float), f)
    np.testing.assert_allclose(p1, p0, atol=1e-13 * f0.sum())


def test_uniform_flow_fixed_point():
    u = np.array([0.05, 0.0, 0.0])
    faces = [INFLOW_EQ, OUTFLOW_ZG, FREESLIP, FREESLIP, FREESLIP, FREESLIP]
    o = oracle.Oracle(12, 6, 5, faces, tau0=0.52, c_smag=0.1, inflow={0: np.tile(u, (5, 1))})
    f0 = o.init(u0=u, amp=0.0)
    np.testing.assert_allclose(f0[:, 2, 3, 4], oracle.equilibrium(1.0, u), rtol=1e-16)
    f = o.run(f0, 30)
    assert np.abs(f - f0).max() <= 1e-15


def test_force_plug_flow_momentum():
    c, _, _ = oracle.lattice()
    F = np.array([2e-6, 0.0, 0.0])
    o = oracle.Oracle(6, 7, 5, [PERIODIC, PERIODIC, FREESLIP, FREESLIP, FREESLIP, FREESLIP],
                      tau0=0.55, c_smag=0.1, force=F)
    f = o.init(amp=0.0)
    n = 6 * 7 * 5
    for t in range(1, 11):
        f = o.step(f)
        p = np.einsum("ia,izyx->a", c.astype(float), f)
        # round-off: ~19 n populations of O(0.1) summed, relative to the total mass n
        np.testing.assert_allclose(p, n * t * F, rtol=0, atol=1e-15 * n)
    # plug flow: every cell moves at the same velocity
    _, u, _ = o.macros(f)
    assert np.ptp(u[0]) < 1e-15


# ---------------------------------------------------------------- streaming
def _frozen(faces, solid, nx=7, ny=6, nz=5):
    # tau0 huge: omega = 1/tau rounds the relaxation away, so a step is pure streaming
    return oracle.Oracle(nx, ny, nz, faces, tau0=1e300, c_smag=0.0, solid=solid)


@pytest.mark.parametrize("faces", [
    [WALL, WALL, WALL, WALL, WALL, WALL],
    [PERIODIC, PERIODIC, FREESLIP, FREESLIP, WALL, FREESLIP],
    [FREESLIP, FREESLIP, FREESLIP, FREESLIP, FREESLIP, FREESLIP],
    [PERIODIC, PERIODIC, PERIODIC, PERIODIC, PERIODIC, PERIODIC],
])
def test_streaming_is_reversible_permutation(faces):
    """In a closed box streaming permutes the populations of the fluid cells,
    and streaming, reversing every direction, streaming again and reversing
    back restores the state exactly (time reversal of the boundary rules)."""
    solid = np.zeros((5, 6, 7), np.uint8)
    solid[0:2, 2:4, 2:4] = 1
    solid[3, 1, 5] = 1
    o = _frozen(faces, solid)
    _, _, opp = oracle.lattice()
    rng = np.random.default_rng(0)
    f0 = rng.random((19, 5, 6, 7))
    f0[:, solid.astype(bool)] = 0.0
    f1 = o.step(f0)
    fluid = ~solid.astype(bool)
    assert np.array_equal(np.sort(f1[:, fluid].ravel()), np.sort(f0[:, fluid].ravel()))
    back = o.step(f1[opp])[opp]
    assert np.array_equal(back[:, fluid], f0[:, fluid])


def test_outflow_copies_inner_layer():
    """Zero-gradient outflow: populations entering through x+ and y+ equal what
    the cell one layer inward (diagonally at the corner) receives."""
    solid = np.zeros((5, 6, 7), np.uint8)
    solid[0:2, 2, 5] = 1     # a solid cell next to the x+ layer
    faces = [INFLOW_EQ, OUTFLOW_ZG, INFLOW_EQ, OUTFLOW_ZG, WALL, FREESLIP]
    prof = np.tile([0.04, 0.02, 0.0], (5, 1))
    o = oracle.Oracle(7, 6, 5, faces, tau0=0.6, c_smag=0.1, solid=solid, inflow={0: prof, 2: prof})
    c, _, opp = oracle.lattice()
    f = o.run(o.init(u0=[0.04, 0.02, 0], amp=1e-3, seed=2), 3)
    fs_prev = None
    nx, ny, nz = 7, 6, 5
    checked = 0
    for z in range(nz):
        for y in range(1, ny):
            x = nx - 1
            if solid[z, y, x]:
                continue
            for i in range(19):
                if c[i, 0] != -1:
                    continue
                xp = [x - 1, y, z]
                if y == ny - 1 and c[i, 1] == -1:
                    xp[1] = y - 1
                if solid[xp[2], xp[1], xp[0]]:
                    continue
                assert f[i, z, y, x] == f[i, xp[2], xp[1], xp[0]]
                checked += 1
    assert checked > 50
    # inflow cells hold the inflow equilibrium
    np.testing.assert_allclose(f[:, 2, 3, 0], oracle.equilibrium(1.0, prof[0]), rtol=1e-16)


# ---------------------------------------------------------------- closed-form flows
def _poiseuille(tau0, ny, steps, g=1e-6):
    nu = (tau0 - 0.5) / 3.0
    eta = np.arange(ny) + 0.5
    exact = g * eta * (ny - eta) / (2.0 * nu)
    o = oracle.Oracle(3, ny, 3, [PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC],
                      tau0=tau0, c_smag=0.0, force=(g, 0, 0))
    u0 = np.zeros((3, 3))
    f = np.zeros((19, 3, ny, 3))
    for y in range(ny):
        f[:, :, y, :] = oracle.equilibrium(1.0, [exact[y], 0, 0])[:, None, None]
    f = o.run(f, steps)
    _, u, _ = o.macros(f)
    return u[0, 1, :, 1], exact


def test_poiseuille_exact_at_magic_tau():
    """Halfway bounce-back places the wall exactly half-way for the BGK
    relaxation time with (tau - 1/2)^2 = 3/16."""
    tau = 0.5 + math.sqrt(3.0) / 4.0
    u, exact = _poiseuille(tau, 16, 6000)
    assert np.abs(u - exact).max() <= 1e-9 * exact.max()


def test_poiseuille_second_order():
    errs = []
    for ny in (8, 16, 32):
        u, exact = _poiseuille(0.6, ny, 40 * ny * ny // 8, g=1e-6 * (8.0 / ny) ** 2)
        errs.append(np.abs(u - exact).max() / exact.max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def _taylor_green(n, tau0, steps, c_smag=0.0, amp=0.01, nz=3):
    k = 2 * math.pi / n
    x = np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")     # [y, x]
    ux = -amp * np.cos(k * X) * np.sin(k * Y)
    uy = amp * np.sin(k * X) * np.cos(k * Y)
    o = oracle.Oracle(n, n, nz, [PERIODIC] * 6, tau0=tau0, c_smag=c_smag)
    f = np.zeros((19, nz, n, n))
    for y in range(n):
        for xx in range(n):
            f[:, :, y, xx] = oracle.equilibrium(1.0, [ux[y, xx], uy[y, xx], 0])[:, None]
    return o, f, (np.cos(k * X) * np.sin(k * Y)), k


def _tg_nu(n, tau0, t0, t1):
    o, f, mode, k = _taylor_green(n, tau0, 0)
    f = o.run(f, t0)
    a0 = -(o.macros(f)[1][0, 1] * mode).sum() / (mode ** 2).sum()
    f = o.run(f, t1 - t0)
    a1 = -(o.macros(f)[1][0, 1] * mode).sum() / (mode ** 2).sum()
    return math.log(a0 / a1) / (2 * k * k * (t1 - t0))


def test_taylor_green_viscosity():
    tau0 = 0.8
    nu = (tau0 - 0.5) / 3.0
    nu64 = _tg_nu(64, tau0, 50, 450)
    assert abs(nu64 / nu - 1.0) < 0.01
    e16 = abs(_tg_nu(16, tau0, 4, 30) / nu - 1)
    e32 = abs(_tg_nu(32, tau0, 12, 112) / nu - 1)
    e64 = abs(nu64 / nu - 1)
    assert e16 / e32 > 3.0 and e32 / e64 > 3.0


def test_smagorinsky_matches_fd_strain():
    """nu_t from the local non-equilibrium closure against (C Delta)^2 |S| with
    the strain rate from central differences of the computed velocity."""
    # tau0 = 0.6 lets the start-up non-equilibrium transient (factor |1 - 1/tau|
    # per step) die out; the remaining gap is the O(h^2) error of the differences
    n, c_smag = 64, 0.2
    o, f, mode, k = _taylor_green(n, 0.6, 0, c_smag=c_smag, amp=0.04)
    f = o.run(f, 60)
    _, u, nut = o.macros(f)
    ux, uy = u[0, 1], u[1, 1]

    def d(a, axis):
        return (np.roll(a, -1, axis) - np.roll(a, 1, axis)) / 2.0

    sxx, syy = d(ux, 1), d(uy, 0)
    sxy = 0.5 * (d(ux, 0) + d(uy, 1))
    smag = np.sqrt(2 * (sxx ** 2 + syy ** 2 + 2 * sxy ** 2))
    ref = c_smag ** 2 * smag
    sel = smag > 0.5 * smag.max()
    rel = np.abs(nut[1][sel] - ref[sel]) / ref[sel]
    assert rel.max() < 0.01
