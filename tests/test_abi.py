"""Host-side checks of the C ABI: the library loads and exports every entry
point include/lbm.h declares; the binding's structs match the header layout."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_2607_04516_amd", "liblbm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("lbm_create", "lbm_set_inflow", "lbm_step", "lbm_macros", "lbm_probe", "lbm_adjoint_step",
              "lbm_mass", "lbm_get_state", "lbm_set_state", "lbm_destroy", "lbm_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_symbol():
    from paper_2607_04516_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_binding_constants_match_header():
    from paper_2607_04516_amd import binding
    src = open(HEADER).read()
    assert int(re.search(r"#define LBM_PROBE_NOALLOC_MAX (\d+)", src).group(1)) == binding.LBM_PROBE_NOALLOC_MAX
    assert int(re.search(r"#define LBM_EINVAL \((-\d+)\)", src).group(1)) == binding.LBM_EINVAL


def test_params_struct_layout():
    from paper_2607_04516_amd import binding
    P = binding._Params
    assert P.tau0.offset == 0 and P.body_force.offset == 32 and P.u_init.offset == 56
    assert P.noise_amp.offset == 80 and P.noise_seed.offset == 88 and P.storage.offset == 96
    assert P.face.offset == 100 and P.watchdog_stride.offset == 124 and P.hip_stream.offset == 128
    assert ctypes.sizeof(P) == 136


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")
def test_params_struct_layout_matches_compiler(tmp_path):
    """Compile a host program against the header and compare offsetof()."""
    import subprocess
    src = tmp_path / "off.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", offsetof(lbm_params,tau0),'
                   'offsetof(lbm_params,body_force), offsetof(lbm_params,u_init), offsetof(lbm_params,noise_amp),'
                   'offsetof(lbm_params,noise_seed), offsetof(lbm_params,storage), offsetof(lbm_params,face),'
                   'offsetof(lbm_params,hip_stream), sizeof(lbm_params)); return 0;}\n')
    exe = tmp_path / "off"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert [int(v) for v in out] == [0, 32, 56, 80, 88, 96, 100, 128, 136]


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblbm.so not built")
def test_turbulence_struct_layout_matches_compiler(tmp_path):
    import subprocess
    from paper_2607_04516_amd import binding
    T = binding._Turbulence
    src = tmp_path / "tu.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu\\n", offsetof(lbm_turbulence,shared),'
                   'offsetof(lbm_turbulence,length_scale), offsetof(lbm_turbulence,sigma0),'
                   'offsetof(lbm_turbulence,gain), offsetof(lbm_turbulence,origin), offsetof(lbm_turbulence,seed),'
                   'sizeof(lbm_turbulence)); return 0;}\n')
    exe = tmp_path / "tu"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).decode().split()]
    assert out == [T.shared.offset, T.length_scale.offset, T.sigma0.offset, T.gain.offset, T.origin.offset,
                   T.seed.offset, ctypes.sizeof(T)]


def test_earth_rotation_vector():
    """App. E: Omega_ENU = Omega (0, cos phi, sin phi), times dt, in grid axes."""
    from paper_2607_04516_amd.binding import OMEGA_EARTH, earth_rotation
    lat, dt = 23.113, 0.01
    om = earth_rotation(lat, dt)
    p = np.radians(lat)
    np.testing.assert_allclose(om, [0.0, OMEGA_EARTH * dt * np.cos(p), OMEGA_EARTH * dt * np.sin(p)], rtol=1e-15)
    # Coriolis parameter f = 2 Omega sin phi (per time step)
    assert abs(2 * om[2] - 2 * OMEGA_EARTH * np.sin(p) * dt) <= 1e-22
    # grid x turned to point north: the horizontal component lies on grid x
    r = earth_rotation(lat, dt, grid_angle_deg=90.0)
    np.testing.assert_allclose(r, [om[1], 0.0, om[2]], atol=1e-20)
    # a small turn (meridian convergence) keeps the magnitude and the vertical part
    r = earth_rotation(lat, dt, grid_angle_deg=-0.911)
    assert abs(np.linalg.norm(r) - OMEGA_EARTH * dt) <= 1e-20 and r[2] == om[2]
    assert r[0] < 0.0    # grid x turned clockwise from east has a southward part
    # the header's constant, and the argument checks
    src = open(HEADER).read()
    assert float(re.search(r"#define LBM_OMEGA_EARTH ([0-9.e-]+)", src).group(1)) == OMEGA_EARTH
    from paper_2607_04516_amd.binding import LBMError
    for bad in ((91.0, 0.01), (23.0, 0.0), (float("nan"), 0.01)):
        with pytest.raises(LBMError):
            earth_rotation(*bad)
