"""Coriolis source on the GPU (App. E) against the oracle and closed forms (needs an MI355X)."""
import math

import numpy as np
import pytest
import torch

from helpers import fluid_mask, oracle_for, oracle_init, small_workload
from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

OMEGA = (0.0, 2e-3, 4e-3)   # large enough that the force shows in every population


def _say(*a):
    print(*a, flush=True)


def _state(lat):
    st, t = lat.get_state()
    torch.cuda.synchronize()
    return lat.state_to_f64(st)


def _solid(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    s = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    s[0, :, : nx // 3] = 0
    return s


@pytest.mark.parametrize("faces", [
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("periodic", "periodic", "periodic", "periodic", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
])
@pytest.mark.parametrize("dims", [(9, 7, 5), (70, 6, 5)])
def test_rotation_stepwise_f64(faces, dims):
    nx, ny, nz = dims
    _say(f"case: coriolis f64 faces {faces} dims {dims}")
    w = small_workload(nx, ny, nz, faces, solid=_solid(nx, ny, nz, nx + ny), omega=OMEGA)
    o = oracle_for(w)
    fo = oracle_init(o, w)
    lat = binding.from_workload(w)
    m = ~w.solid.astype(bool)
    for step in range(1, 7):
        fo = o.step(fo)
        lat.step(1)
        fg = _state(lat)
        d = np.abs(fg - fo)[:, m] / np.abs(fo[:, m])
        assert d.max() <= 1e-12, f"step {step}: {d.max()}"


@pytest.mark.parametrize("storage,bar", [("f32", 2e-5), ("f16s", 5e-4)])
def test_rotation_cube_reduced_precision(storage, bar):
    w = workloads.cube_flow(storage, 100)
    w.omega = OMEGA
    o = oracle_for(w)
    fo = o.run(oracle_init(o, w), 100)
    _, uo, _ = o.macros(fo)
    lat = binding.from_workload(w)
    lat.step(100)
    rho, u, _ = lat.macros()
    torch.cuda.synchronize()
    ug = u.double().cpu().numpy()
    m = ~w.solid.astype(bool)
    err = np.abs(ug - uo)[:, m].max()
    _say(f"{storage} + rotation: max |du| {err:.2e}")
    assert err <= bar


def test_inertial_oscillation_f32():
    """Uniform flow in a periodic box turns at exactly m -> (I + f J) m per step."""
    f_cor = 2e-3
    nx, ny, nz = 130, 6, 5
    w = small_workload(nx, ny, nz, ["periodic"] * 6, tau0=0.55, c_smag=0.1, u=(0.05, 0.0, 0.0),
                       noise=0.0, storage="f32", omega=(0.0, 0.0, f_cor / 2))
    lat = binding.from_workload(w)
    steps = 400
    lat.step(steps)
    _, u, _ = lat.macros()
    torch.cuda.synchronize()
    ug = u.double().cpu().numpy().reshape(3, -1).mean(axis=1)
    amp = 0.05 * (1 + f_cor ** 2) ** (steps / 2)
    ang = -steps * math.atan(f_cor)
    # reported u = (m + F/2)/rho: half a step of the rotation ahead of m
    mx, my = amp * math.cos(ang), amp * math.sin(ang)
    want = np.array([mx + 0.5 * f_cor * my, my - 0.5 * f_cor * mx, 0.0])
    assert np.abs(ug - want).max() <= 1e-6


def test_zero_rotation_bit_identical():
    w = small_workload(70, 6, 5, ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
                       solid=_solid(70, 6, 5, 1), storage="f32")
    a = binding.from_workload(w)
    b = binding.from_workload(w)
    b.set_rotation((0.0, 0.0, 0.0))
    a.step(9)
    b.step(9)
    sa, _ = a.get_state()
    sb, _ = b.get_state()
    torch.cuda.synchronize()
    assert torch.equal(sa, sb)


def test_rotation_push_chain_bit_exact():
    w = workloads.adjoint_urban("f32", 20, small=True)
    w.omega = OMEGA
    lat = binding.from_workload(w)
    s0, _ = lat.get_state()
    s0 = s0.clone()
    lat.step(20)
    ref, _ = lat.get_state()
    a, b = s0.clone(), lat.new_state()
    for _ in range(20):
        lat.push_step(a, b)
        a, b = b, a
    torch.cuda.synchronize()
    assert torch.equal(a, ref)


@pytest.mark.parametrize("faces", [
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
])
def test_rotation_adjoint_step_f64(faces):
    nx, ny, nz = 11, 8, 6
    rng = np.random.default_rng(3)
    solid = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8)
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.15, u=(0.05, 0.02, 0.01),
                       noise=5e-3, seed=4, force=(2e-5, 0.0, 0.0), omega=OMEGA)
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    probes = np.argwhere(m)[:: max(1, m.sum() // 5)][:5][:, ::-1].astype(np.int32)
    src = rng.standard_normal((len(probes), 3))
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lat = binding.from_workload(w)
    lat.set_probes(probes)
    ft = lat.f64_to_state(f)
    ln = torch.from_numpy(lam_next).to("cuda", torch.float64).contiguous()
    lam = torch.empty_like(ln)
    ps = torch.from_numpy(src).to("cuda", torch.float64).contiguous()
    g = torch.zeros(2, 6, nz, 3, dtype=torch.float64, device="cuda")
    lat.adjoint_step(ft, ln, lam, ps, g)
    torch.cuda.synchronize()
    lam_g = lam.cpu().numpy()
    g_g = (g[0] + g[1]).cpu().numpy()
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * np.abs(lam_o).max()
    assert np.abs(g_g - g_o).max() <= 1e-12 * np.abs(g_o).max()


def test_set_rotation_rejects_bad_input():
    w = small_workload(9, 7, 5, ["periodic"] * 6)
    lat = binding.from_workload(w)
    for bad in [(0.0, float("nan"), 0.0), (0.3, 0.0, 0.0), (0.0, 0.0, float("inf"))]:
        with pytest.raises(binding.LBMError):
            lat.set_rotation(bad)
    lat.set_rotation((0.0, 1e-3, 2e-3))
    lat.step(2)
