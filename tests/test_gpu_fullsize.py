"""Full-size parity on the benchmark workload (needs an MI355X).

800 x 800 x 128 urban grid (the configuration bench.py times), run a few
steps, export f(t), take one more step on the GPU, and recompute f(t+1) of
sampled cells one by one with the oracle's window step (FP64): random
interior cells, every face layer and corner, cells next to buildings.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import oracle_for, window_index
from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")

W_ = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _samples(w, rng, n_random=1500):
    nx, ny, nz = w.nx, w.ny, w.nz
    s = w.solid.astype(bool)
    pts = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(n_random)]
    for _ in range(60):   # every face layer
        y, z, x = int(rng.integers(ny)), int(rng.integers(nz)), int(rng.integers(nx))
        pts += [(0, y, z), (nx - 1, y, z), (x, 0, z), (x, ny - 1, z), (x, y, 0), (x, y, nz - 1)]
    for x in (0, 1, nx - 2, nx - 1):   # edges and corners
        for y in (0, 1, ny - 2, ny - 1):
            for z in (0, 1, nz - 2, nz - 1):
                pts.append((x, y, z))
    # fluid cells next to buildings
    zz, yy, xx = np.nonzero(s[:-1] & ~s[1:])
    k = rng.choice(len(zz), size=min(300, len(zz)), replace=False)
    pts += [(int(xx[i]), int(yy[i]), int(zz[i] + 1)) for i in k]
    pts = [p for p in dict.fromkeys(pts) if not s[p[2], p[1], p[0]]]
    return np.array(pts, np.int64)


def _windows(state, pts, faces, nx, ny, nz):
    zi, yi, xi = (torch.from_numpy(a).to(state.device) for a in window_index(pts, faces, nx, ny, nz))
    win = state[:, zi, yi, xi]            # [19, S, 5, 5, 5]
    return win.permute(1, 0, 2, 3, 4).contiguous()


@pytest.mark.parametrize("t0", [10, 11])
@pytest.mark.parametrize("storage,bar", [("f64", 1e-12), ("f32", 1e-6), ("f16s", None)])
def test_fullsize_sampled_cells(storage, bar, t0):
    """From an even time the next launch is the even (local) kernel, from an
    odd time the odd (gather) kernel."""
    print(f"case: urban_km 800x800x128 {storage}, sampled one-step parity from t = {t0}", flush=True)
    w = workloads.urban_km(storage, 12)
    lat = binding.from_workload(w)
    lat.step(t0)
    ft, t = lat.get_state()
    ft = ft.clone()
    lat.step(1)
    fn, _ = lat.get_state()
    torch.cuda.synchronize()
    pts = _samples(w, np.random.default_rng(1))
    win = _windows(ft, pts, w.faces, w.nx, w.ny, w.nz).to(torch.float64).cpu().numpy() / lat.scale
    win += W_[None, :, None, None, None]
    got = fn[:, pts[:, 2], pts[:, 1], pts[:, 0]].to(torch.float64).cpu().numpy().T / lat.scale + W_
    o = oracle_for(w)
    worst = 0.0
    for k, (x, y, z) in enumerate(pts):
        ref = o.step_cell(win[k], int(x), int(y), int(z))
        if bar is None:
            # binary16 storage: one rounding of 256 h, half an ulp of 2^-11 relative
            tol = 2.0 ** -11 * np.abs(ref - W_) + 2e-7
            assert np.all(np.abs(got[k] - ref) <= tol), (x, y, z)
        else:
            err = np.abs(got[k] - ref).max() / np.abs(ref).max()
            worst = max(worst, err)
            assert err <= bar, (x, y, z, err)
    print(f"{storage}: {len(pts)} cells, worst relative error {worst:.2e}", flush=True)


def test_fullsize_eight_slabs_bit_identical():
    """The kilometre grid as eight 800 x 100 x 128 slabs (ghost rows and halo
    exchange, one per rank of an eight-GPU run) on this GPU matches the
    whole-grid run bit for bit."""
    print("case: urban_km 800x800x128 f32 as 8 slabs", flush=True)
    from paper_2607_04516_amd import slabs
    w = workloads.urban_km("f32", 12)
    whole = binding.from_workload(w)
    dec = slabs.SlabDecomposition(w, 8)
    s0, _ = whole.get_state()
    dec.set_state(s0, 0)
    del s0
    whole.step(5)
    dec.step(5)
    ref, _ = whole.get_state()
    got = dec.get_state()
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    dec.close()
    whole.close()
