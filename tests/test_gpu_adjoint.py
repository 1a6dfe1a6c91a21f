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


X_EDGE_FACES = [
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
    ("inflow", "outflow", "periodic", "periodic", "freeslip", "outflow"),
]


@pytest.mark.parametrize("fi", range(len(X_EDGE_FACES)))
@pytest.mark.parametrize("dims", [(5, 6, 5), (65, 5, 4), (66, 5, 4), (130, 4, 5)])
def test_adjoint_step_x_face_lanes_f64(fi, dims):
    """The x-face layers of an inflow/outflow pair inside the adjoint's waves:
    solids in and next to both face columns (bounce-back into and out of the
    outflow copies, solid inflow cells), face columns on either side of a
    64-cell chunk boundary."""
    print(f"case: adjoint x-face lanes faces {X_EDGE_FACES[fi]} dims {dims}", flush=True)
    nx, ny, nz = dims
    rng = np.random.default_rng(31 + fi + nx)
    solid = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    for cols in ((0, 1, 2), (nx - 3, nx - 2, nx - 1)):
        for x in cols:
            solid[:, :, x] |= (rng.random((nz, ny)) < 0.3).astype(np.uint8)
    w = small_workload(nx, ny, nz, X_EDGE_FACES[fi], solid=solid, tau0=0.53, c_smag=0.15,
                       u=(0.05, 0.02, 0.01), noise=5e-3, seed=fi + 40)
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    probes = np.argwhere(m)[:: max(1, m.sum() // 5)][:5][:, ::-1].astype(np.int32)
    src = rng.standard_normal((len(probes), 3))
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    err = np.abs(lam_g - lam_o)
    assert err.max() <= 1e-12 * np.abs(lam_o).max(), np.argwhere(err > 1e-12 * np.abs(lam_o).max())[:6].tolist()
    assert np.abs(g_g - g_o).max() <= 1e-12 * max(np.abs(g_o).max(), 1e-30)


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


def test_adjoint_probe_sources_every_path_f64():
    """Probe sources added inside the adjoint kernel: probes in several 64-cell
    chunks of the interior waves and in the face shell, repeated probes of one
    cell, and probes on solid and inflow cells (no source), with rotation on so
    that the Coriolis part of du/df enters."""
    nx, ny, nz = 140, 7, 6
    rng = np.random.default_rng(21)
    solid = (rng.random((nz, ny, nx)) < 0.06).astype(np.uint8)
    solid[:, :, :3] = 0
    solid[:, :, nx - 3:] = 0
    solid[2, 3, 70] = 1
    w = small_workload(nx, ny, nz, ("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
                       solid=solid, tau0=0.53, c_smag=0.15, u=(0.05, 0.02, 0.01), noise=5e-3, seed=13,
                       omega=(1e-4, 2e-4, -3e-4))
    o = oracle_for(w)
    f = o.run(oracle_init(o, w), 3)
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    cells = [(5, 3, 2), (63, 1, 4), (64, 1, 4), (100, 5, 1), (127, 2, 3), (128, 2, 3), (135, 6, 5),
             (1, 2, 2), (nx - 2, 4, 1), (0, 3, 3), (nx - 1, 3, 3), (70, 3, 2), (64, 1, 4), (64, 1, 4),
             (1, 2, 2), (33, 0, 0), (90, 6, 5)]
    probes = np.array(cells, np.int32)
    src = rng.standard_normal((len(probes), 3))
    print(f"case: adjoint probe sources, {len(probes)} probes on {nx}x{ny}x{nz}", flush=True)
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    assert np.abs(lam_g - lam_o).max() <= 1e-12 * np.abs(lam_o).max()
    assert np.abs(g_g - g_o).max() <= 1e-12 * np.abs(g_o).max()
    # the sources themselves: the same step without them differs exactly at the probe cells
    lam_0, _ = o.adjoint_step(f, lam_next)
    moved = np.abs(lam_o - lam_0).max(axis=0) > 0
    want = np.zeros_like(moved)
    for x, y, z in cells:
        if m[z, y, x] and x != 0:
            want[z, y, x] = True
    assert np.array_equal(moved, want)


def test_push_step_matches_forward_with_inflow_faces_f32():
    """The push recompute (face-layer blocks plus interior waves in one
    launch) against the in-place forward step, bit for bit, on a grid with
    INFLOW faces on x-, y- and z+ (interior pushes next to them are skipped)."""
    nx, ny, nz = 140, 9, 8
    rng = np.random.default_rng(5)
    solid = (rng.random((nz, ny, nx)) < 0.06).astype(np.uint8)
    w = small_workload(nx, ny, nz, ("inflow", "outflow", "inflow", "outflow", "wall", "inflow"), solid=solid,
                       tau0=0.53, c_smag=0.15, u=(0.05, 0.02, 0.0), noise=5e-3, seed=3, storage="f32")
    lat = binding.from_workload(w)
    s0, _ = lat.get_state()
    a, b = s0.clone(), lat.new_state()
    for step in range(6):
        lat.step(1)
        ref, _ = lat.get_state()
        lat.push_step(a, b)
        a, b = b, a
        torch.cuda.synchronize()
        assert torch.equal(a, ref), step


@pytest.mark.parametrize("fi", range(len(X_EDGE_FACES)))
@pytest.mark.parametrize("dims", [(5, 6, 5), (65, 5, 4), (66, 5, 4), (130, 4, 5)])
def test_push_step_x_face_cells(fi, dims):
    """The push recompute with the x-face cells of an inflow/outflow pair
    inside its waves: FP64 against the oracle step, FP32 bit for bit against
    the in-place forward step, with solids in and next to both face columns."""
    print(f"case: push x-face cells faces {X_EDGE_FACES[fi]} dims {dims}", flush=True)
    nx, ny, nz = dims
    rng = np.random.default_rng(57 + fi + nx)
    solid = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    for x in (0, 1, 2, nx - 3, nx - 2, nx - 1):
        solid[:, :, x] |= (rng.random((nz, ny)) < 0.3).astype(np.uint8)
    for storage in ("f64", "f32", "f16s"):
        w = small_workload(nx, ny, nz, X_EDGE_FACES[fi], solid=solid, tau0=0.53, c_smag=0.15,
                           u=(0.05, 0.02, 0.01), noise=5e-3, seed=fi + 60, storage=storage)
        lat = binding.from_workload(w)
        if storage == "f64":
            o = oracle_for(w)
            f0 = o.run(oracle_init(o, w), 3)
            f1 = o.step(f0)
            dst = lat.new_state()
            lat.push_step(lat.f64_to_state(f0), dst)
            torch.cuda.synchronize()
            fg = lat.state_to_f64(dst)
            m = ~w.solid.astype(bool)
            scale = np.abs(f1[:, m]).max()
            assert np.abs(fg[:, m] - f1[:, m]).max() <= 1e-12 * scale
        else:
            s0, _ = lat.get_state()
            a, b = s0.clone(), lat.new_state()
            for step in range(4):
                lat.step(1)
                ref, _ = lat.get_state()
                lat.push_step(a, b)
                a, b = b, a
                torch.cuda.synchronize()
                assert torch.equal(a, ref), step
        lat.close()


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
@pytest.mark.parametrize("fi", [0, 1])
def test_adjoint_step_16bit_snapshots(storage, fi):
    """The adjoint with 16-bit stored states (FP32 arithmetic): against the
    oracle adjoint at the same decoded state, to the FP32 bar."""
    print(f"case: adjoint {storage} faces {X_EDGE_FACES[fi]}", flush=True)
    nx, ny, nz = 66, 6, 5
    rng = np.random.default_rng(71 + fi)
    solid = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    w = small_workload(nx, ny, nz, X_EDGE_FACES[fi], solid=solid, tau0=0.53, c_smag=0.15,
                       u=(0.05, 0.02, 0.01), noise=5e-3, seed=fi + 80, storage=storage)
    o = oracle_for(w)
    lat = binding.from_workload(w)
    f = lat.state_to_f64(lat.f64_to_state(o.run(oracle_init(o, w), 3)))   # the state the GPU sees
    lat.close()
    m = fluid_mask(w)
    lam_next = rng.standard_normal(f.shape) * m[None]
    probes = np.argwhere(m)[:: max(1, m.sum() // 5)][:5][:, ::-1].astype(np.int32)
    src = rng.standard_normal((len(probes), 3))
    lam_o, g_o = o.adjoint_step(f, lam_next, probes, src)
    lam_g, g_g = _gpu_adjoint(w, f, lam_next, probes, src)
    err = np.abs(lam_g - lam_o).max() / np.abs(lam_o).max()
    gerr = np.abs(g_g - g_o).max() / np.abs(g_o).max()
    print(f"{storage} adjoint relative errors: lam {err:.2e}, g {gerr:.2e}", flush=True)
    assert err <= 2e-5 and gerr <= 2e-5
