"""The watchdog's unstable case on the oracle (no GPU): the 32x24x16 cube
channel with tau0 just above 1/2, no eddy viscosity and inflow at 0.25 leaves
the stable range within the first 200 steps in FP64 too, so the GPU's
EUNSTABLE there is the method's instability, not an artefact of the device
arithmetic; the stable configuration of the same grid stays bounded."""
import numpy as np

from helpers import oracle_for, oracle_init
from paper_2607_04516_amd import workloads


def _cube_small(tau0, u, c_smag):
    nx, ny, nz = 32, 24, 16
    solid = workloads.cube_mask(nx, ny, nz, x0=8, size=(4, 4, 6))
    prof = workloads.uniform_profile(nz, (u, 0.0, 0.0))
    return workloads.Workload("cube_small", nx, ny, nz, workloads.FACES_CHANNEL, tau0, c_smag, "f64", 10, solid,
                              {0: prof}, prof.copy(), noise_seed=1)


def _first_unstable_step(w, steps, stride=10):
    """First multiple of stride at which the watchdog's test fails (non-finite
    values, max |u|^2 > 0.25 or max |rho - rho0| > 0.5 over fluid cells), or None."""
    o = oracle_for(w)
    f = oracle_init(o, w)
    fluid = ~w.solid.astype(bool)
    for t in range(1, steps + 1):
        f = o.step(f)
        if t % stride:
            continue
        rho, u, _ = o.macros(f)
        r = rho[fluid]
        u2 = (u * u).sum(0)[fluid]
        if not (np.all(np.isfinite(r)) and np.all(np.isfinite(u2))):
            return t
        if np.max(u2) > 0.25 or np.max(np.abs(r - 1.0)) > 0.5:
            return t
    return None


def test_unstable_configuration_fails_on_the_oracle():
    t = _first_unstable_step(_cube_small(0.5001, 0.25, 0.0), 200)
    assert t is not None and t <= 200


def test_stable_configuration_stays_bounded_on_the_oracle():
    assert _first_unstable_step(_cube_small(0.52, 0.05, 0.1), 200) is None
