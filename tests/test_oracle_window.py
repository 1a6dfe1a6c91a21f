"""Pin of the oracle's one-cell window step against its full step.

The window step (f(x, t+1) of one cell from the 5x5x5 window of f(t) around
it) is the reference of the full-size GPU parity test, which samples cells of
a grid too large for a full oracle step.  Here it must reproduce the full
oracle step bit for bit at every non-solid cell of small grids, with the
windows built by the rule the GPU test uses (tests/helpers.window_index):
every face set of the boundary matrix (inflow/outflow corners, two inflow
faces, periodic wraps, solids on faces), plus the sponge, Earth rotation, a
body force, per-cell face states and a per-cell inflow velocity field.
"""
import numpy as np
import pytest

import oracle
from helpers import FACE_SETS, FACE_NUM, windows_np


def _solid(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    s = (rng.random((nz, ny, nx)) < 0.12).astype(np.uint8)
    s[nz // 2, :, 0] = 1           # solids on faces and edges
    s[:, -1, nx - 1] = 1
    s[0, 0, :] = 1
    return s


def _random_state(o, seed):
    """A non-trivial state: a noisy start, two steps, then independent noise
    on every population so that no two window entries coincide."""
    rng = np.random.default_rng(seed)
    f = o.run(o.init(u0=[0.04, 0.01, -0.005], amp=2e-3, seed=seed), 2)
    return f + 2e-3 * rng.standard_normal(f.shape) * (o.solid == 0)[None]


def _check_all_cells(o, faces, f):
    nz, ny, nx = o.shape
    ref = o.step(f)
    pts = np.array([(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)
                    if not o.solid[z, y, x]], np.int64)
    win = windows_np(f, pts, faces, nx, ny, nz)
    for k, (x, y, z) in enumerate(pts):
        got = o.step_cell(win[k], int(x), int(y), int(z))
        np.testing.assert_array_equal(got, ref[:, z, y, x], err_msg=f"cell {(x, y, z)} faces {faces}")
    return len(pts)


def _uniform_inflow(faces, nz, rng):
    prof = np.array([0.04, 0.01, 0.0]) + 0.005 * rng.standard_normal((nz, 3))
    return {k: prof.copy() for k, f in enumerate(faces) if f == "inflow"}


@pytest.mark.parametrize("fi", range(len(FACE_SETS)))
@pytest.mark.parametrize("dims", [(5, 4, 6), (9, 7, 4), (12, 6, 5)])
def test_window_step_equals_full_step(fi, dims):
    faces = FACE_SETS[fi]
    nx, ny, nz = dims
    rng = np.random.default_rng(fi * 10 + nx)
    o = oracle.Oracle(nx, ny, nz, [FACE_NUM[f] for f in faces], tau0=0.53, c_smag=0.15,
                      solid=_solid(nx, ny, nz, fi + nx), inflow=_uniform_inflow(faces, nz, rng))
    n = _check_all_cells(o, faces, _random_state(o, fi + 3))
    assert n > 0.6 * nx * ny * nz


SPECIAL = [
    # sponge / buffer layers next to three inflow faces, the top one included
    dict(faces=("inflow", "outflow", "inflow", "freeslip", "wall", "inflow"), sponge=(2, 0.2)),
    # Earth rotation (Coriolis through the Guo source) and a uniform body force
    dict(faces=("inflow", "outflow", "freeslip", "freeslip", "wall", "freeslip"),
         omega=(0.0, 2e-3, 4e-3), force=(1e-5, -2e-6, 0.0)),
    # per-cell boundary states on three faces
    dict(faces=("inflow", "outflow", "inflow", "outflow", "wall", "inflow"), arrays=True, sponge=(2, 0.1)),
    # per-cell inflow velocity field (the synthetic-inflow form), periodic y
    dict(faces=("inflow", "outflow", "periodic", "periodic", "wall", "freeslip"), field=True),
]


@pytest.mark.parametrize("case", range(len(SPECIAL)))
def test_window_step_special_terms(case):
    c = SPECIAL[case]
    faces = c["faces"]
    nx, ny, nz = 11, 7, 6
    rng = np.random.default_rng(100 + case)
    inflow = _uniform_inflow(faces, nz, rng)
    if c.get("arrays"):
        for k in list(inflow):
            n2, n1 = oracle.face_shape(k, nx, ny, nz)
            inflow[k] = np.array([0.04, 0.01, 0.0]) + 0.01 * rng.standard_normal((n2, n1, 3))
    o = oracle.Oracle(nx, ny, nz, [FACE_NUM[f] for f in faces], tau0=0.54, c_smag=0.12,
                      solid=_solid(nx, ny, nz, 40 + case), inflow=inflow, omega=c.get("omega", (0, 0, 0)),
                      force=c.get("force", (0, 0, 0)), sponge=c.get("sponge", (0, 0.0)))
    if c.get("field"):
        o.inflow_field = np.array([0.05, 0.0, 0.0]) + 0.01 * rng.standard_normal((nz, ny, nx, 3))
    _check_all_cells(o, faces, _random_state(o, 7 + case))


def test_window_transpose_is_detected():
    """A window with its x and y axes exchanged (the mistake a wrong index
    order in the window step would make) changes the result."""
    faces = FACE_SETS[2]
    nx, ny, nz = 9, 7, 4
    o = oracle.Oracle(nx, ny, nz, [FACE_NUM[f] for f in faces], tau0=0.53, c_smag=0.15,
                      solid=_solid(nx, ny, nz, 3), inflow=_uniform_inflow(faces, nz, np.random.default_rng(0)))
    f = _random_state(o, 1)
    ref = o.step(f)
    x, y, z = 4, 3, 2
    win = windows_np(f, np.array([[x, y, z]]), faces, nx, ny, nz)[0]
    assert np.array_equal(o.step_cell(win, x, y, z), ref[:, z, y, x])
    assert not np.array_equal(o.step_cell(np.swapaxes(win, 2, 3).copy(), x, y, z), ref[:, z, y, x])
