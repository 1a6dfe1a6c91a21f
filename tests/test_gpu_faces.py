"""Per-cell boundary states of the INFLOW_EQ faces (lbm_set_inflow_face) on
the GPU against the oracle (needs an MI355X): inflow cells, sponge targets at
the cell's projection, flux balancing, the synthetic inflow's mean field and
the adjoint's inflow gradient all read the per-cell states."""
import numpy as np
import pytest
import torch

from helpers import FACE_NUM, fluid_mask, oracle_for, oracle_init, small_workload
from oracle import face_shape
from oracle import stabilize as st
from oracle import vk

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

FACES = ("inflow", "outflow", "inflow", "freeslip", "wall", "inflow")


def _say(*a):
    print(*a, flush=True)


def _state(lat):
    s, _ = lat.get_state()
    torch.cuda.synchronize()
    return lat.state_to_f64(s)


def _workload(nx=70, ny=10, nz=9, storage="f64", sponge=(3, 0.25), seed=3, faces=FACES):
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.05).astype(np.uint8)
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.12, u=(0.04, 0.01, 0.0),
                       noise=3e-3, seed=seed, storage=storage)
    for f in list(w.inflow):
        n2, n1 = face_shape(f, nx, ny, nz)
        w.inflow[f] = np.array([0.04, 0.012, -0.002]) + rng.normal(0.0, 0.008, (n2, n1, 3))
    w.sponge = sponge
    return w


@pytest.mark.parametrize("dims", [(9, 8, 7), (70, 10, 9)])
def test_face_states_stepwise_f64(dims):
    nx, ny, nz = dims
    _say(f"case: per-cell face states f64 {dims}")
    w = _workload(nx, ny, nz)
    o = oracle_for(w)
    fo = oracle_init(o, w)
    lat = binding.from_workload(w)
    for f, arr in w.inflow.items():
        got = lat.get_inflow(f)
        np.testing.assert_array_equal(got.reshape(arr.shape), arr)
    m = ~w.solid.astype(bool)
    for step in range(1, 6):
        fo = o.step(fo)
        lat.step(1)
        fg = _state(lat)
        err = (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max()
        assert err <= 1e-12, (step, err)


def test_face_states_f32_80_steps():
    w = _workload(storage="f32")
    o = oracle_for(w)
    fo = o.run(oracle_init(o, w), 80)
    _, uo, _ = o.macros(fo)
    lat = binding.from_workload(w)
    lat.step(80)
    _, u, _ = lat.macros()
    torch.cuda.synchronize()
    err = np.abs(u.double().cpu().numpy() - uo)[:, ~w.solid.astype(bool)].max()
    _say(f"f32 per-cell face states: max |du| {err:.2e}")
    assert err <= 2e-5


def test_profile_replaces_face_states():
    w = _workload(sponge=(0, 0.0))
    lat = binding.from_workload(w)
    prof = np.tile([0.03, 0.0, 0.0], (w.nz, 1))
    lat.set_inflow(0, prof)
    got = lat.get_inflow(0).reshape(face_shape(0, w.nx, w.ny, w.nz) + (3,))
    np.testing.assert_array_equal(got, np.broadcast_to(prof[:, None, :], got.shape))
    with pytest.raises(binding.LBMError):
        lat.set_inflow(1, w.inflow[0])          # x+ is not an inflow face
    bad = w.inflow[2].copy()
    bad[1, 1, 0] = np.nan
    with pytest.raises(binding.LBMError):
        lat.set_inflow(2, bad)


def test_flux_balance_of_face_states():
    faces = ("inflow", "inflow", "inflow", "inflow", "wall", "inflow")
    w = _workload(faces=faces, sponge=(0, 0.0), seed=7)
    fn = [FACE_NUM[f] for f in faces]
    lat = binding.from_workload(w)
    before, after = lat.balance_flux(1)
    arr_o, phi_o, _ = st.balance_profiles(fn, w.solid, w.inflow)
    assert abs(before - phi_o) <= 1e-13 * max(1.0, abs(phi_o))
    assert abs(after) <= 1e-12 and abs(lat.net_flux()) <= 1e-12
    for f, arr in arr_o.items():
        np.testing.assert_allclose(lat.get_inflow(f).reshape(arr.shape), arr, rtol=0, atol=1e-16)
    w.inflow = arr_o
    o = oracle_for(w)
    fo = o.run(oracle_init(o, w), 4)
    lat.reset(w.u0)
    lat.step(4)
    fg = _state(lat)
    m = ~w.solid.astype(bool)
    assert (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max() <= 1e-12


def test_turbulence_around_face_states():
    w = _workload(sponge=(0, 0.0), seed=9)
    fn = [FACE_NUM[f] for f in w.faces]
    kw = dict(n_modes=12, length_scale=4.0, intensity=0.2, seed=6)
    lat = binding.from_workload(w)
    lat.set_turbulence(**kw)
    gen = vk.VonKarmanInflow(fn, w.solid, w.inflow, vk.VKParams(**kw))
    n, u_ref, _ = lat.turbulence_info()
    assert n == len(gen.cells) and abs(u_ref - gen.u_ref) <= 1e-15
    lat.reset(w.u0)
    o = oracle_for(w)
    o.inflow_field = gen.field(0)
    fo = oracle_init(o, w)
    m = ~w.solid.astype(bool)
    for t in range(4):
        o.inflow_field = gen.field(t)
        fo = o.step(fo)
        lat.step(1)
        fg = _state(lat)
        err = (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max()
        assert err <= 1e-12, (t, err)


def test_adjoint_inflow_gradient_with_face_states_f64():
    """Each inflow cell's own velocity enters d feq/du; the per-height
    gradient sums over the row."""
    w = _workload(nx=70, ny=8, nz=7, sponge=(0, 0.0), seed=11)
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    rng = np.random.default_rng(2)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    lam_o, g_o = o.adjoint_step(f, lam_next)
    lat = binding.from_workload(w)
    rd = lat.real_dtype
    ft = lat.f64_to_state(f)
    ln = torch.from_numpy(lam_next).to("cuda", rd).contiguous()
    lam = torch.empty_like(ln)
    g = torch.zeros(2, 6, w.nz, 3, dtype=rd, device="cuda")
    lat.adjoint_step(ft, ln, lam, None, g)
    torch.cuda.synchronize()
    lam_g = lam.double().cpu().numpy()
    g_g = (g[0] + g[1]).double().cpu().numpy()
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * np.abs(lam_o).max()
    assert np.abs(g_g - g_o).max() <= 1e-12 * np.abs(g_o).max()
