"""Open-boundary stabilisers on the GPU against the oracle (needs an MI355X):
sponge / buffer nudging inside the step kernels, global flux balancing of
the profiles and of the per-cell boundary field."""
import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_init, small_workload
from oracle import stabilize as st
from oracle import vk
from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

FACE_NUM = {"periodic": 0, "inflow": 1, "outflow": 2, "freeslip": 3, "wall": 4}


def _say(*a):
    print(*a, flush=True)


def _state(lat):
    s, _ = lat.get_state()
    torch.cuda.synchronize()
    return lat.state_to_f64(s)


def _workload(faces, nx=70, ny=10, nz=9, storage="f64", sponge=(3, 0.25), seed=2):
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.05).astype(np.uint8)
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.12, u=(0.04, 0.01, 0.0),
                       noise=3e-3, seed=seed, storage=storage)
    prof = workloads.direction_profile(workloads.power_law_speeds(nz, 0.06, 6.0, 0.25), 0.3)
    for k in w.inflow:
        w.inflow[k] = prof.copy()
    w.sponge = sponge
    return w


SPONGE_FACES = [
    ("inflow", "outflow", "inflow", "outflow", "wall", "inflow"),
    ("inflow", "inflow", "inflow", "inflow", "wall", "inflow"),
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
]


@pytest.mark.parametrize("faces", SPONGE_FACES)
@pytest.mark.parametrize("dims", [(9, 8, 9), (70, 10, 9)])
def test_sponge_stepwise_f64(faces, dims):
    nx, ny, nz = dims
    _say(f"case: sponge f64 faces {faces} dims {dims}")
    w = _workload(faces, nx, ny, nz)
    o = oracle_for(w)
    fo = oracle_init(o, w)
    lat = binding.from_workload(w)
    m = ~w.solid.astype(bool)
    for step in range(1, 7):
        fo = o.step(fo)
        lat.step(1)
        fg = _state(lat)
        err = (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max()
        assert err <= 1e-12, (step, err)


@pytest.mark.parametrize("storage,bar", [("f32", 2e-5), ("f16s", 5e-4)])
def test_sponge_reduced_precision(storage, bar):
    w = _workload(SPONGE_FACES[0], storage=storage, sponge=(4, 0.3))
    o = oracle_for(w)
    fo = o.run(oracle_init(o, w), 80)
    _, uo, _ = o.macros(fo)
    lat = binding.from_workload(w)
    lat.step(80)
    _, u, _ = lat.macros()
    torch.cuda.synchronize()
    err = np.abs(u.double().cpu().numpy() - uo)[:, ~w.solid.astype(bool)].max()
    _say(f"{storage} + sponge: max |du| {err:.2e}")
    assert err <= bar


def test_sponge_push_chain_bit_exact_and_adjoint_refused():
    w = _workload(SPONGE_FACES[0], storage="f32")
    lat = binding.from_workload(w)
    s0, _ = lat.get_state()
    s0 = s0.clone()
    lat.step(12)
    ref, _ = lat.get_state()
    a, b = s0.clone(), lat.new_state()
    for _ in range(12):
        lat.push_step(a, b)
        a, b = b, a
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
    lam = torch.zeros(19, w.nz, w.ny, w.nx, dtype=torch.float32, device="cuda")
    g = torch.zeros(2, 6, w.nz, 3, dtype=torch.float32, device="cuda")
    with pytest.raises(binding.LBMError):
        lat.adjoint_step(ref, lam, torch.empty_like(lam), None, g)
    lat.set_sponge(0, 0.0)
    lat.adjoint_step(ref, lam, torch.empty_like(lam), None, g)


def test_sponge_rejects_bad_input():
    w = _workload(SPONGE_FACES[0], sponge=(0, 0.0))
    lat = binding.from_workload(w)
    for wd, s in [(-1, 0.1), (3, 1.5), (3, -0.1), (200, 0.1), (3, float("nan"))]:
        with pytest.raises(binding.LBMError):
            lat.set_sponge(wd, s)


OPEN = ("inflow", "inflow", "inflow", "inflow", "wall", "inflow")


def _imbalanced(storage="f64"):
    w = _workload(OPEN, storage=storage, sponge=(0, 0.0))
    nz = w.nz
    w.inflow[1] = np.tile([0.03, 0.0, 0.0], (nz, 1))       # x+ face: slower, leaving the domain
    w.inflow[3] = np.tile([0.01, 0.02, 0.0], (nz, 1))
    w.inflow[5] = np.tile([0.05, 0.0, -0.004], (nz, 1))
    return w


def test_flux_balance_profiles_matches_oracle():
    w = _imbalanced()
    faces = [FACE_NUM[f] for f in w.faces]
    lat = binding.from_workload(w)
    before, after = lat.balance_flux(1)
    prof_o, phi_o, after_o = st.balance_profiles(faces, w.solid, w.inflow)
    assert abs(before - phi_o) <= 1e-13 * abs(phi_o)
    assert abs(after) <= 1e-12 * abs(phi_o) and abs(after_o) <= 1e-12 * abs(phi_o)
    # the device field now equals the balanced profiles, and its flux is ~0
    for face in (0, 1, 2, 3, 5):
        got = lat.get_inflow(face)
        a = face // 2
        z = np.arange(w.nz) if a < 2 else np.full(w.ny, w.nz - 1)
        want = prof_o[face][z]
        np.testing.assert_allclose(got.reshape(-1, got.shape[-2], 3)[:, 0], want, atol=1e-16)
    assert abs(lat.net_flux()) <= 1e-12 * abs(phi_o)
    # and the run matches the oracle on the balanced profiles
    w.inflow = prof_o
    o = oracle_for(w)
    fo = o.run(oracle_init(o, w), 5)
    lat.reset(w.u0)
    lat.step(5)
    fg = _state(lat)
    m = ~w.solid.astype(bool)
    assert (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max() <= 1e-12


def test_flux_balance_every_step_with_turbulence():
    """Mode 2: the full field (profiles plus synthetic turbulence) is balanced
    on the device before every step; the oracle balances its field the same way."""
    w = _imbalanced()
    faces = [FACE_NUM[f] for f in w.faces]
    kw = dict(n_modes=16, length_scale=5.0, intensity=0.2, seed=4)
    lat = binding.from_workload(w)
    lat.set_turbulence(**kw)
    lat.balance_flux(2)
    lat.reset(w.u0)
    gen = vk.VonKarmanInflow(faces, w.solid, w.inflow,
                             vk.VKParams(n_modes=16, length_scale=5.0, intensity=0.2, seed=4))
    o = oracle_for(w)
    o.inflow_field = gen.field(0)          # reset: the generator's field, not yet balanced
    fo = oracle_init(o, w)
    m = ~w.solid.astype(bool)
    for t in range(6):
        fld, phi, after = st.balance_field(faces, w.solid, gen.field(t))
        o.inflow_field = fld
        fo = o.step(fo)
        lat.step(1)
        assert abs(lat.net_flux()) <= 1e-12 * abs(phi)
        fg = _state(lat)
        err = (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max()
        assert err <= 1e-12, (t, err)
    lat.balance_flux(0)
