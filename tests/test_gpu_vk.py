"""Synthetic von Karman inflow on the GPU (App. F) against the oracle (needs an MI355X)."""
import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_init, small_workload
from oracle import vk
from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

FACES = ("inflow", "outflow", "inflow", "outflow", "wall", "inflow")


def _say(*a):
    print(*a, flush=True)


def _workload(nx=70, ny=9, nz=7, storage="f64", faces=FACES, seed=3):
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.06).astype(np.uint8)
    solid[:, 0, 5:8] = 1                      # solid cells on the y- inflow face
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.12, u=(0.05, 0.02, 0.0),
                       noise=2e-3, seed=seed, storage=storage)
    # a sheared profile, so sigma and the face means vary with height
    prof = workloads.direction_profile(workloads.power_law_speeds(nz, 0.06, 5.0, 0.25), 0.35)
    prof[:, 2] = 0.004 * np.sin(np.arange(nz))
    for k in w.inflow:
        w.inflow[k] = prof.copy()
    w.u0 = prof.copy()
    return w


def _params(**kw):
    base = dict(n_modes=24, length_scale=6.0, intensity=0.2, seed=11)
    base.update(kw)
    return base


def _oracle_gen(w, kw, origin=(0, 0, 0)):
    faces = [{"inflow": 1, "outflow": 2, "freeslip": 3, "wall": 4, "periodic": 0}[f] for f in w.faces]
    p = vk.VKParams(n_modes=kw["n_modes"], length_scale=kw["length_scale"], intensity=kw.get("intensity", 0.1),
                    sigma0=kw.get("sigma0", 0.0), gains=kw.get("gains", (1.0, 1.0, 1.0)),
                    char_normal=kw.get("char_normal", False), inflow_only=kw.get("inflow_only", False),
                    shared=kw.get("shared", False), stride=kw.get("stride", 1),
                    interpolate=kw.get("interpolate", False), seed=kw["seed"], origin=origin)
    return vk.VonKarmanInflow(faces, w.solid, w.inflow, p)


def _face_values(field, face, nx, ny, nz):
    a = face // 2
    if a == 0:
        return field[:, :, 0 if face == 0 else nx - 1]
    if a == 1:
        return field[:, 0 if face == 2 else ny - 1, :]
    return field[0 if face == 4 else nz - 1]


def _owned(w, face):
    """Non-solid cells whose inflow face is this one (a cell on two inflow
    faces belongs to the lower-numbered face)."""
    faces = [{"inflow": 1, "outflow": 2, "freeslip": 3, "wall": 4, "periodic": 0}[f] for f in w.faces]
    own = np.zeros(w.solid.shape, bool)
    for z in range(w.nz):
        for y in range(w.ny):
            for x in range(w.nx):
                own[z, y, x] = not w.solid[z, y, x] and vk.owner_face(faces, w.nx, w.ny, w.nz, x, y, z) == face
    return own


CASES = {
    "plain": {},
    "hold": dict(stride=4),
    "interp": dict(stride=4, interpolate=True),
    "shared_gains": dict(shared=True, gains=(1.0, 0.5, 0.25)),
    "normal_filter": dict(char_normal=True, inflow_only=True),
    "sigma0": dict(intensity=0.0, sigma0=0.003),
}


@pytest.mark.parametrize("case", list(CASES))
def test_boundary_field_matches_oracle(case):
    _say(f"case: von Karman field {case}")
    w = _workload()
    kw = _params(**CASES[case])
    lat = binding.from_workload(w)
    origin = (5.0, -3.0, 2.0)
    lat.set_turbulence(origin=origin, **kw)
    lat.reset(w.u0)
    gen = _oracle_gen(w, kw, origin)
    n, u_ref, e_c = lat.turbulence_info()
    assert n == len(gen.cells)
    assert abs(u_ref - gen.u_ref) <= 1e-13 * gen.u_ref
    np.testing.assert_allclose(e_c, gen.e_c, atol=1e-14)
    for t in (0, 1, 2, 5, 9):
        if t:
            lat.step(t - lat.time + 1)     # the last step started from time t
        fo = gen.field(t)
        for face in (0, 2, 5):
            got = lat.get_inflow(face)
            want = _face_values(fo, face, w.nx, w.ny, w.nz)
            keep = _face_values(_owned(w, face)[..., None].repeat(3, -1), face, w.nx, w.ny, w.nz)
            d = np.abs(got - want)[keep]
            assert d.max() <= 1e-13, (t, face, d.max())


def test_stepwise_f64_with_turbulence():
    w = _workload()
    kw = _params(stride=3, interpolate=True)
    gen = _oracle_gen(w, kw)
    o = oracle_for(w)
    o.inflow_field = gen.field(0)
    fo = oracle_init(o, w)
    lat = binding.from_workload(w)
    lat.set_turbulence(**kw)
    lat.reset(w.u0)
    m = ~w.solid.astype(bool)
    for t in range(8):
        o.inflow_field = gen.field(t)
        fo = o.step(fo)
        lat.step(1)
        st, _ = lat.get_state()
        torch.cuda.synchronize()
        fg = lat.state_to_f64(st)
        err = (np.abs(fg - fo)[:, m] / np.abs(fo[:, m])).max()
        assert err <= 1e-12, (t, err)


@pytest.mark.parametrize("storage,bar", [("f32", 2e-5), ("f16s", 5e-4)])
def test_reduced_precision_velocity_with_turbulence(storage, bar):
    w = _workload(storage=storage)
    kw = _params()
    gen = _oracle_gen(w, kw)
    o = oracle_for(w)
    o.inflow_field = gen.field(0)
    fo = oracle_init(o, w)
    for t in range(60):
        o.inflow_field = gen.field(t)
        fo = o.step(fo)
    _, uo, _ = o.macros(fo)
    lat = binding.from_workload(w)
    lat.set_turbulence(**kw)
    lat.reset(w.u0)
    lat.step(60)
    _, u, _ = lat.macros()
    torch.cuda.synchronize()
    err = np.abs(u.double().cpu().numpy() - uo)[:, ~w.solid.astype(bool)].max()
    _say(f"{storage} + turbulence: max |du| {err:.2e}")
    assert err <= bar


def test_profile_change_rebuilds_and_off_restores():
    w = _workload()
    lat = binding.from_workload(w)
    lat.set_turbulence(**_params())
    n0, u0, _ = lat.turbulence_info()
    lat.set_inflow(0, 2.0 * w.inflow[0])
    n1, u1, _ = lat.turbulence_info()
    assert n1 == n0 and u1 > u0
    s0, _ = lat.get_state()
    with pytest.raises(binding.LBMError):
        lat.push_step(s0.clone(), lat.new_state())
    lat.set_turbulence(enable=False)
    assert lat.turbulence_info()[0] == 0
    lat.set_inflow(0, w.inflow[0])
    np.testing.assert_array_equal(lat.get_inflow(0)[:, :, :], np.broadcast_to(w.inflow[0][:, None, :],
                                                                                (w.nz, w.ny, 3)))
    lat.push_step(s0.clone(), lat.new_state())


def test_bad_parameters_rejected():
    w = _workload()
    lat = binding.from_workload(w)
    for bad in [dict(n_modes=0), dict(n_modes=5000), dict(stride=0), dict(length_scale=0.0),
                dict(intensity=float("nan"))]:
        with pytest.raises(binding.LBMError):
            lat.set_turbulence(**_params(**bad))
    assert lat.turbulence_info()[0] == 0
