"""Slab decomposition along y with ghost rows and halo exchange, emulated on
one GPU (needs an MI355X): the slabs reproduce the undecomposed run bit for
bit, in every storage codec, with buildings crossing the interfaces, inflow
and outflow on the slab-crossing faces, the sponge and rotation on."""
import numpy as np
import pytest
import torch

from helpers import small_workload
from oracle import face_shape

pytestmark = pytest.mark.gpu

binding = pytest.importorskip("paper_2607_04516_amd.binding")
slabs = pytest.importorskip("paper_2607_04516_amd.slabs")

FACE_SETS = [
    ("inflow", "outflow", "inflow", "outflow", "wall", "freeslip"),
    ("inflow", "outflow", "freeslip", "freeslip", "wall", "inflow"),
    ("periodic", "periodic", "wall", "outflow", "periodic", "periodic"),
]


def _say(*a):
    print(*a, flush=True)


def _workload(faces, storage, nx=70, ny=23, nz=9, seed=4):
    rng = np.random.default_rng(seed)
    solid = (rng.random((nz, ny, nx)) < 0.08).astype(np.uint8)
    solid[: nz // 2, 5:11, 20:26] = 1            # a building across the first interface (y = 8)
    solid[2:5, 14:17, 40:44] = 1                 # and one across the second (y = 15)
    w = small_workload(nx, ny, nz, faces, solid=solid, tau0=0.53, c_smag=0.12, u=(0.04, 0.012, 0.0),
                       noise=3e-3, seed=seed, storage=storage, omega=(1e-4, 3e-4, 5e-4))
    for f in list(w.inflow):
        n2, n1 = face_shape(f, nx, ny, nz)
        w.inflow[f] = np.array([0.04, 0.012, 0.0]) + rng.normal(0.0, 0.006, (n2, n1, 3))
    w.sponge = (2, 0.2)
    return w


@pytest.mark.parametrize("fi", range(len(FACE_SETS)))
@pytest.mark.parametrize("storage", ["f32", "f64", "f16s"])
def test_slabs_reproduce_the_whole_grid_bit_for_bit(fi, storage):
    _say(f"case: halo slabs faces {FACE_SETS[fi]} {storage}")
    w = _workload(FACE_SETS[fi], storage)
    whole = binding.from_workload(w)
    dec = slabs.SlabDecomposition(w, 3)
    s0, _ = whole.get_state()
    dec.set_state(s0.clone(), 0)
    for step in range(1, 11):
        whole.step(1)
        dec.step(1)
        ref, _ = whole.get_state()
        got = dec.get_state()
        torch.cuda.synchronize()
        if not torch.equal(got, ref):
            bad = (got != ref).nonzero()
            raise AssertionError(f"step {step}: {bad.shape[0]} entries differ, first {bad[:5].tolist()}")
    dec.close()
    whole.close()


def test_uneven_slabs_and_thin_slab():
    w = _workload(FACE_SETS[0], "f32", ny=20)
    whole = binding.from_workload(w)
    dec = slabs.SlabDecomposition(w, 3, rows=[(0, 3), (3, 15), (15, 20)])
    s0, _ = whole.get_state()
    dec.set_state(s0.clone(), 0)
    whole.step(7)
    dec.step(7)
    ref, _ = whole.get_state()
    torch.cuda.synchronize()
    assert torch.equal(dec.get_state(), ref)


def test_halo_faces_refuse_what_needs_all_slabs():
    w = _workload(FACE_SETS[0], "f32")
    dec = slabs.SlabDecomposition(w, 2)
    lat = dec.slabs[0]
    buf = lat.halo_buffer()
    with pytest.raises(binding.LBMError):
        lat.halo_pack(0, buf)                     # y- of the first slab is the domain's face
    with pytest.raises(binding.LBMError):
        lat.set_turbulence(n_modes=8)
    with pytest.raises(binding.LBMError):
        lat.balance_flux(2)
    s, _ = lat.get_state()
    with pytest.raises(binding.LBMError):
        lat.push_step(s, lat.new_state())
    with pytest.raises(binding.LBMError):
        binding.LBM(8, 8, 8, faces=("halo", "outflow", "wall", "wall", "wall", "wall"))
    dec.close()
