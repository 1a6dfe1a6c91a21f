"""lbm_probe_noalloc against lbm_probe (needs an MI355X).

The no-allocation probe entry point stages points and results through the
library's fixed per-GPU scratch array; it must return exactly what lbm_probe
returns (same kernel, same inputs), on two calls in a row, the second with
fewer points, and refuse more points than the scratch holds.
"""
import numpy as np
import pytest
import torch

from paper_2607_04516_amd import workloads

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")


def _points(w, n, seed):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.uniform(0, w.nx - 1, n), rng.uniform(0, w.ny - 1, n), rng.uniform(0, w.nz - 1, n)], axis=1)
    pts[: n // 4] = np.round(pts[: n // 4])   # integer points return the cell itself
    return pts.astype(np.float32)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_probe_noalloc_matches_probe(storage):
    w = workloads.urban_subdomain(storage, 30)
    print(f"case: lbm_probe_noalloc vs lbm_probe, urban subdomain 128x128x64 {storage}", flush=True)
    lat = binding.from_workload(w)
    lat.step(31)   # odd time: the swapped layout
    for n, seed in ((binding.LBM_PROBE_NOALLOC_MAX, 1), (1000, 2)):
        pts = _points(w, n, seed)
        ref = lat.probe(pts)
        got = lat.probe_noalloc(pts)
        torch.cuda.synchronize()
        assert got.shape == ref.shape == (n, 4)
        assert np.array_equal(got, ref), (n, np.abs(got - ref).max())
        assert np.isfinite(got).all()
    lat.step(1)    # even time: natural layout
    pts = _points(w, 77, 3)
    assert np.array_equal(lat.probe_noalloc(pts), lat.probe(pts))
    with pytest.raises(binding.LBMError) as exc:
        lat.probe_noalloc(_points(w, binding.LBM_PROBE_NOALLOC_MAX + 1, 4))
    assert exc.value.code == binding.LBM_EINVAL
    lat.close()
