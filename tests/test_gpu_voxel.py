"""The ray-parity voxelizer on the GPU (needs an MI355X): the same labels as
the oracle, bit for bit, on closed-form solids, rotated buildings, ties and
a leaking mesh; the urban building boxes reproduce the height-map mask at
full size."""
import math
import time

import numpy as np
import pytest

from oracle import voxel
from paper_2607_04516_amd import workloads as W

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")


def _cases():
    yield "box", (20, 22, 70), [W.box_mesh(3, 11, 4, 17, 0, 9), W.box_mesh(60, 69, 2, 20, 3, 18)]
    yield "octahedron", (21, 23, 25), [W.octahedron_mesh(11.3, 10.7, 9.2, 6.13)]
    yield "prisms", (20, 22, 130), [W.prism_mesh(12.1 + 25 * k, 10.9, 11.0, 6.0, 0.3 + 0.7 * k, 0.0, 13.7)
                                    for k in range(5)]
    yield "cavity", (20, 22, 24), [W.box_mesh(2, 12, 2, 12, 0, 10), W.box_mesh(8, 20, 6, 18, 0, 14),
                                   np.concatenate([W.box_mesh(1, 23, 1, 21, 12, 19),
                                                   W.box_mesh(5, 9, 5, 9, 14, 17)[:, ::-1]])]
    yield "half_integer", (20, 22, 24), [W.box_mesh(3.5, 10.5, 4.5, 12.5, 2.5, 9.5)]
    yield "leak", (20, 22, 24), [W.box_mesh(4, 14, 5, 15, 2, 12)[1:]]
    rng = np.random.default_rng(3)
    tets = []
    for _ in range(6):
        v = rng.uniform(0.7, 19.3, (4, 3))
        tets.append(np.array([[v[0], v[1], v[2]], [v[0], v[1], v[3]], [v[0], v[2], v[3]], [v[1], v[2], v[3]]]))
    yield "tetrahedra", (21, 20, 22), tets
    yield "rotated_city", (40, 90, 131), W.rotated_building_meshes(131, 90, 40, 11, hmax=35.0, margin=2.0)


@pytest.mark.parametrize("passes", [1, 3])
@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_labels_match_the_oracle(case, passes):
    name, shape, meshes = case
    print(f"case: voxelize {name} {shape} passes {passes}", flush=True)
    t, s = W.meshes_to_arrays(meshes)
    base = np.zeros(shape, np.uint8)
    base[0, :2, :] = 1                                    # something to OR into
    want = voxel.voxelize(shape, t, s, passes, solid=base)
    got = binding.voxelize(shape, t, s, passes, solid=base)
    np.testing.assert_array_equal(got, want)


def test_urban_boxes_give_the_height_map_mask_at_full_size():
    nx, ny, nz = 800, 800, 128
    meshes = W.urban_box_meshes(nx, ny, 0.30, 12, 0.5, 100, 5, (10, 40), 32, 32)
    t, s = W.meshes_to_arrays(meshes)
    want = W.heights_to_mask(W.urban_heights(nx, ny, 0.30, 12, 0.5, 100, 5, (10, 40), 32, 32), nz)
    for passes in (1, 3):
        t0 = time.perf_counter()
        got = binding.voxelize((nz, ny, nx), t, s, passes)
        dt = time.perf_counter() - t0
        print(f"urban_km buildings: {len(meshes)} meshes, {len(t)} triangles, {passes} pass(es): {dt * 1e3:.1f} ms",
              flush=True)
        np.testing.assert_array_equal(got, want)


def test_bad_input_is_refused():
    t, s = W.meshes_to_arrays([W.box_mesh(1, 3, 1, 3, 1, 3)])
    with pytest.raises(binding.LBMError):
        binding.voxelize((8, 8, 8), t, s, passes=2)
    with pytest.raises(binding.LBMError):
        binding.voxelize((8, 8, 8), t, np.array([0, 5], np.int32))
    bad = t.copy()
    bad[0, 0, 0] = math.nan
    with pytest.raises(binding.LBMError):
        binding.voxelize((8, 8, 8), bad, s)
    with pytest.raises(binding.LBMError):
        binding.voxelize((2000, 8, 8), t, s)          # a ray longer than 1024 cells
