"""GPU discrete-adjoint step against the FP64 oracle adjoint (needs an MI355X).

The GPU applies the transposed streaming as a gather and the collision
transpose matrix-free; the oracle scatter-adds over every pull and multiplies
by an explicit 19x19 Jacobian.  Both see the same canonical state and the
same lam_next; lam(t) and the inflow-profile gradient are compared.
"""
import numpy as np
import pytest
import torch

from helpers import fluid_mask, oracle_for, oracle_init, small_workload

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

FACE_SETS = [
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
    ("periodic", "periodic", "wall", "outflow", "freeslip", "outflow"),
    ("outflow", "inflow", "outflow", "outflow", "freeslip", "outflow"),
    ("wall", "wall", "periodic", "periodic", "wall", "freeslip"),
]


def _problem(fi, dims, storage, seed=0, force=(0.0, 0.0, 0.0)):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed + fi)
    solid = (rng.random((nz, ny, nx)) < 0.1).astype(np.uint8)
    w = small_workload(nx, ny, nz, FACE_SETS[fi], solid=solid, tau0=0.53, c_smag=0.15,
                       u=(0.05, 0.02, 0.01), noise=5e-3, seed=seed + 4, storage=storage, force=force)
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    probes = np.argwhere(m)[:: max(1, m.sum() // 5)][:5][:, ::-1].astype(np.int32)   # (x, y, z)
    src = rng.standard_normal((len(probes), 3))
    return w, o, f, lam_next, probes, src


def _gpu_adjoint(w, f, lam_next, probes, src):
    lat = binding.from_workload(w)
    lat.set_probes(probes)
    rd = lat.real_dtype
    ft = lat.f64_to_state(f)
    ln = torch.from_numpy(lam_next).to("cuda", rd).contiguous()
    lam = torch.empty_like(ln)
    ps = torch.from_numpy(src).to("cuda", rd).contiguous()
    g = torch.zeros(2, 6, w.nz, 3, dtype=rd, device="cuda")
    lat.adjoint_step(ft, ln, lam, ps, g)
    torch.cuda.synchronize()
    return lam.double().cpu().numpy(), (g[0] + g[1]).double().cpu().numpy()


@pytest.mark.parametrize("fi", range(len(FACE_SETS)))
@pytest.mark.parametrize("dims", [(7, 6, 5), (11, 8, 6)])
def test_adjoint_step_f64_matches_oracle(fi, dims):
    print(f"case: adjoint f64 faces {FACE_SETS[fi]} dims {dims}", flush=True)
    w, o, f, lam_next, probes, src = _problem(fi, dims, "f64")
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    scale = np.abs(lam_o).max()
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * scale
    gs = max(np.abs(g_o).max(), 1e-30)
    assert np.abs(g_g - g_o).max() <= 1e-12 * gs


def test_adjoint_step_freeslip_rows_multichunk_f64():
    """Free-slip face rows in the fast adjoint kernel, several chunks, solids in the face rows."""
    nx, ny, nz = 140, 7, 6
    rng = np.random.default_rng(11)
    solid = (rng.random((nz, ny, nx)) < 0.05).astype(np.uint8)
    for x in (5, 63, 64, 100, 127, 128):
        solid[2, 0, x] = solid[3, ny - 1, x] = solid[nz - 1, 3, x] = 1
    solid[:, :, :3] = 0
    solid[:, :, nx - 3:] = 0
    w = small_workload(nx, ny, nz, ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
                       solid=solid, tau0=0.53, c_smag=0.15, u=(0.05, 0.02, 0.01), noise=5e-3, seed=9)
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    probes = np.argwhere(m)[:: max(1, m.sum() // 5)][:5][:, ::-1].astype(np.int32)
    src = rng.standard_normal((len(probes), 3))
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * np.abs(lam_o).max()
    assert np.abs(g_g - g_o).max() <= 1e-12 * np.abs(g_o).max()


def test_adjoint_step_force_f64():
    w, o, f, lam_next, probes, src = _problem(0, (9, 6, 5), "f64", force=(2e-5, -1e-5, 3e-6))
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * np.abs(lam_o).max()
    assert np.abs(g_g - g_o).max() <= 1e-12 * np.abs(g_o).max()


@pytest.mark.parametrize("fi", [0, 1])
def test_adjoint_step_f32(fi):
    w, o, f, lam_next, probes, src = _problem(fi, (12, 9, 7), "f32")
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    err = np.abs(lam_g - lam_o).max() / np.abs(lam_o).max()
    gerr = np.abs(g_g - g_o).max() / np.abs(g_o).max()
    print(f"f32 adjoint relative errors: lam {err:.2e}, g {gerr:.2e}", flush=True)
    assert err <= 2e-5 and gerr <= 2e-5
