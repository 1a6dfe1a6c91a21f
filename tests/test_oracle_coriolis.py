"""Pins of the oracle's Coriolis source (App. E) against rotating-frame physics.

Reading of the sign: the force per unit volume is F = -2 rho Omega x u with
Omega the rotation vector in the east-north-up frame, Omega = |Omega| (0,
cos phi, sin phi) at latitude phi.  Every pin below is stated in a form
other than the cross product the oracle evaluates:

* the component equations of the rotating-frame momentum budget (the f and
  f~ = 2 |Omega| cos phi parameters of dynamic meteorology): an east wind is
  turned to the south and pushed upward in the northern hemisphere;
* inertial oscillation on the f-plane: uniform flow turns clockwise at the
  Coriolis frequency f = 2 |Omega| sin phi, and the explicit Guo step
  advances the momentum by exactly m -> (I + f J) m per step;
* the momentum component along Omega is invariant in a periodic box, for
  any flow (the force is perpendicular to Omega).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import PERIODIC

OMEGA_EARTH = 7.292115e-5   # rad/s (App. E)


def _momentum(f):
    c, _, _ = oracle.lattice()
    return np.einsum("ia,izyx->a", c.astype(float), f)


def _enu(omega, lat_deg):
    p = math.radians(lat_deg)
    return np.array([0.0, omega * math.cos(p), omega * math.sin(p)])


@pytest.mark.parametrize("lat", [23.113, -35.0, 90.0, 0.0])
@pytest.mark.parametrize("u0", [(0.05, 0.0, 0.0), (0.0, 0.04, 0.0), (0.02, -0.03, 0.01)])
def test_coriolis_component_equations(lat, u0):
    """One step from a uniform state: dm = rho (f v - f~ w, -f u, f~ u)."""
    om = 1e-3
    o = oracle.Oracle(4, 4, 4, [PERIODIC] * 6, tau0=0.6, c_smag=0.1, omega=_enu(om, lat))
    f0 = o.init(u0=u0, amp=0.0)
    n = 64
    rho = f0.sum() / n
    dm = (_momentum(o.step(f0)) - _momentum(f0)) / n
    p = math.radians(lat)
    fc, ft = 2 * om * math.sin(p), 2 * om * math.cos(p)
    u, v, w = u0
    want = rho * np.array([fc * v - ft * w, -fc * u, ft * u])
    np.testing.assert_allclose(dm, want, rtol=0, atol=1e-15)


def test_east_wind_turns_south_and_up_in_north():
    o = oracle.Oracle(4, 4, 4, [PERIODIC] * 6, tau0=0.6, omega=_enu(1e-3, 45.0))
    f0 = o.init(u0=(0.05, 0.0, 0.0), amp=0.0)
    dm = _momentum(o.step(f0)) - _momentum(f0)
    assert dm[1] < 0 and dm[2] > 0 and abs(dm[0]) < 1e-13


def test_inertial_oscillation_f_plane():
    """Uniform flow on the f-plane: exact discrete rotation, and the
    continuous clockwise oscillation at frequency f within O(f^2 t)."""
    f_cor = 2e-3
    o = oracle.Oracle(3, 3, 3, [PERIODIC] * 6, tau0=0.55, c_smag=0.1, omega=(0.0, 0.0, f_cor / 2))
    U = 0.05
    f = o.init(u0=(U, 0.0, 0.0), amp=0.0)
    n = 27
    rho = f.sum() / n
    steps = 400
    for _ in range(steps):
        f = o.step(f)
    m = _momentum(f) / n / rho
    # explicit step m -> (I + f J) m, J = [[0, 1], [-1, 0]]: amplitude (1 + f^2)^(k/2), angle -k atan f
    amp = U * (1 + f_cor ** 2) ** (steps / 2)
    ang = -steps * math.atan(f_cor)
    np.testing.assert_allclose(m, [amp * math.cos(ang), amp * math.sin(ang), 0.0], rtol=0, atol=1e-13)
    # continuous inertial oscillation u = U (cos ft, -sin ft)
    t = steps
    cont = np.array([U * math.cos(f_cor * t), -U * math.sin(f_cor * t)])
    assert np.abs(m[:2] - cont).max() <= 2 * f_cor ** 2 * t * U
    assert m[1] < 0    # clockwise in the northern hemisphere


def test_momentum_along_rotation_axis_is_invariant():
    om = _enu(2e-3, 30.0)
    o = oracle.Oracle(7, 6, 5, [PERIODIC] * 6, tau0=0.52, c_smag=0.1, omega=om)
    f0 = o.init(u0=(0.03, -0.02, 0.01), amp=0.02, seed=4)
    p0 = _momentum(f0)
    f = o.run(f0, 40)
    p1 = _momentum(f)
    axis = om / np.linalg.norm(om)
    assert abs(axis @ (p1 - p0)) <= 1e-13 * f0.sum()
    # and the perpendicular part really turned
    assert np.linalg.norm(p1 - p0) > 1e-3 * np.linalg.norm(p0)
    m0, _ = o.mass(f0)
    m1, _ = o.mass(f)
    assert abs(m1 - m0) <= 1e-13 * m0


def test_zero_rotation_is_unchanged():
    a = oracle.Oracle(6, 5, 4, [PERIODIC] * 6, tau0=0.52, c_smag=0.1, force=(1e-6, 0, 0))
    b = oracle.Oracle(6, 5, 4, [PERIODIC] * 6, tau0=0.52, c_smag=0.1, force=(1e-6, 0, 0),
                      omega=(0.0, 0.0, 0.0))
    f0 = a.init(u0=(0.02, 0.01, 0.0), amp=0.01, seed=2)
    assert np.array_equal(a.run(f0, 5), b.run(f0, 5))
