"""ctypes binding of liblbm.so (include/lbm.h).

Argument marshalling only: every step of the update runs in the HIP kernels of
the library.  PyTorch supplies device memory (tensors) and the HIP stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

F64, F32, F16S, BF16S = 0, 1, 2, 3
STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S}
STORE_DTYPE = {F64: torch.float64, F32: torch.float32, F16S: torch.float16, BF16S: torch.bfloat16}
REAL_DTYPE = {F64: torch.float64, F32: torch.float32, F16S: torch.float32, BF16S: torch.float32}
# binary16 storage holds 256 * h (power-of-two scale into the normal range)
STORE_SCALE = {F64: 1.0, F32: 1.0, F16S: 256.0, BF16S: 1.0}

FACE_KIND = {"periodic": 0, "inflow": 1, "outflow": 2, "freeslip": 3, "wall": 4, "halo": 5}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EUNSTABLE", -5: "ESTATE"}
LBM_EINVAL = -1
LBM_PROBE_NOALLOC_MAX = 16384   # include/lbm.h: points per lbm_probe_noalloc call

# D3Q19 weights in the library's direction order (for h <-> f conversions)
WEIGHTS = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("tau0", ctypes.c_double), ("c_smag", ctypes.c_double), ("delta", ctypes.c_double),
                ("rho0", ctypes.c_double), ("body_force", ctypes.c_double * 3),
                ("u_init", ctypes.c_double * 3), ("noise_amp", ctypes.c_double),
                ("noise_seed", ctypes.c_uint64), ("storage", ctypes.c_int32),
                ("face", ctypes.c_int32 * 6), ("watchdog_stride", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p)]


class _Turbulence(ctypes.Structure):
    _fields_ = [("n_modes", ctypes.c_int32), ("stride", ctypes.c_int32), ("interpolate", ctypes.c_int32),
                ("char_normal", ctypes.c_int32), ("inflow_only", ctypes.c_int32), ("shared", ctypes.c_int32),
                ("length_scale", ctypes.c_double), ("intensity", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("gain", ctypes.c_double * 3), ("origin", ctypes.c_double * 3), ("seed", ctypes.c_uint64)]


EXPORTS = ["lbm_create", "lbm_destroy", "lbm_set_inflow", "lbm_set_inflow_face", "lbm_set_rotation",
           "lbm_earth_rotation", "lbm_set_turbulence",
           "lbm_turbulence_info", "lbm_get_inflow", "lbm_set_sponge", "lbm_balance_flux", "lbm_net_flux",
           "lbm_reset", "lbm_step", "lbm_step_probed",
           "lbm_macros", "lbm_probe", "lbm_probe_noalloc", "lbm_mass", "lbm_get_state", "lbm_set_state", "lbm_set_probes",
           "lbm_probe_accumulate", "lbm_set_stats", "lbm_push_step", "lbm_adjoint_step", "lbm_time",
           "lbm_cell_counts", "lbm_layout", "lbm_set_stream", "lbm_last_error", "lbm_profile", "lbm_profile_read",
           "lbm_halo_pack", "lbm_halo_unpack", "lbm_voxelize"]

_lib = None


def load(path: str = LIB_PATH):
    """Load liblbm.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(or python paper_2607_04516_amd/build_lib.py)")
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "lbm_create": ([ctypes.POINTER(_Grid), P, ctypes.POINTER(_Params), ctypes.POINTER(P)], ctypes.c_int),
        "lbm_destroy": ([P], None),
        "lbm_set_inflow": ([P, I32, P], ctypes.c_int),
        "lbm_set_inflow_face": ([P, I32, P], ctypes.c_int),
        "lbm_halo_pack": ([P, I32, P], ctypes.c_int),
        "lbm_voxelize": ([ctypes.POINTER(_Grid), P, I32, P, I32, I32, P], ctypes.c_int),
        "lbm_halo_unpack": ([P, I32, P], ctypes.c_int),
        "lbm_set_rotation": ([P, P], ctypes.c_int),
        "lbm_earth_rotation": ([ctypes.c_double, ctypes.c_double, ctypes.c_double, P], ctypes.c_int),
        "lbm_set_turbulence": ([P, ctypes.POINTER(_Turbulence)], ctypes.c_int),
        "lbm_turbulence_info": ([P, P, P, P], ctypes.c_int),
        "lbm_get_inflow": ([P, I32, P], ctypes.c_int),
        "lbm_set_sponge": ([P, I32, ctypes.c_double], ctypes.c_int),
        "lbm_balance_flux": ([P, I32, P, P], ctypes.c_int),
        "lbm_net_flux": ([P, P], ctypes.c_int),
        "lbm_reset": ([P, P], ctypes.c_int),
        "lbm_step": ([P, I64], ctypes.c_int),
        "lbm_step_probed": ([P, I64, P], ctypes.c_int),
        "lbm_macros": ([P, P, P, P], ctypes.c_int),
        "lbm_probe": ([P, P, I32, P], ctypes.c_int),
        "lbm_probe_noalloc": ([P, P, I32, P], ctypes.c_int),
        "lbm_mass": ([P, P, P], ctypes.c_int),
        "lbm_get_state": ([P, P, ctypes.POINTER(I64)], ctypes.c_int),
        "lbm_set_state": ([P, P, I64], ctypes.c_int),
        "lbm_set_probes": ([P, P, I32], ctypes.c_int),
        "lbm_probe_accumulate": ([P, P], ctypes.c_int),
        "lbm_set_stats": ([P, P, I32], ctypes.c_int),
        "lbm_push_step": ([P, P, P], ctypes.c_int),
        "lbm_adjoint_step": ([P, P, P, P, P, P], ctypes.c_int),
        "lbm_time": ([P], I64),
        "lbm_cell_counts": ([P, P, P], ctypes.c_int),
        "lbm_layout": ([P, P, P, P], ctypes.c_int),
        "lbm_set_stream": ([P, P], ctypes.c_int),
        "lbm_last_error": ([P], ctypes.c_char_p),
        "lbm_profile": ([P, I32], ctypes.c_int),
        "lbm_profile_read": ([P, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr())
    return t


class LBM:
    """One lattice context (owns the device state through liblbm)."""

    def __init__(self, nx, ny, nz, solid=None, faces=("periodic",) * 6, tau0=0.6, c_smag=0.0,
                 delta=1.0, rho0=1.0, force=(0.0, 0.0, 0.0), storage="f32", u_init=(0.0, 0.0, 0.0),
                 noise_amp=0.0, noise_seed=0, watchdog_stride=0, device="cuda", stream=None):
        self.lib = load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.device = torch.device(device)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.store_dtype = STORE_DTYPE[self.storage]
        self.real_dtype = REAL_DTYPE[self.storage]
        self.scale = STORE_SCALE[self.storage]
        self.rho0 = float(rho0)
        if solid is None:
            solid = np.zeros((nz, ny, nx), np.uint8)
        self.solid = np.ascontiguousarray(solid, np.uint8).reshape(nz, ny, nx)
        self.faces = tuple(FACE_KIND[f] if isinstance(f, str) else int(f) for f in faces)
        p = _Params()
        p.tau0, p.c_smag, p.delta, p.rho0 = tau0, c_smag, delta, rho0
        for a in range(3):
            p.body_force[a] = float(force[a])
            p.u_init[a] = float(u_init[a])
        p.noise_amp, p.noise_seed = float(noise_amp), int(noise_seed)
        p.storage = self.storage
        for k in range(6):
            p.face[k] = self.faces[k]
        p.watchdog_stride = int(watchdog_stride)
        if stream is None:
            with torch.cuda.device(self.device):
                stream = torch.cuda.current_stream()
        self.stream = stream
        p.hip_stream = ctypes.c_void_p(stream.cuda_stream)
        g = _Grid(self.nx, self.ny, self.nz)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.lbm_create(ctypes.byref(g), self.solid.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(p), ctypes.byref(ctx))
        if rc != 0:
            raise LBMError(rc, self.lib.lbm_last_error(None).decode())
        self.ctx = ctx
        self.np = 0

    # -- plumbing ---------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise LBMError(rc, self.lib.lbm_last_error(self.ctx).decode())

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls ----------------------------------------------------------
    def face_shape(self, face):
        """(n2, n1) of a face's per-cell arrays: cell (j1, j2) is (y, z) on the
        x faces, (x, z) on the y faces, (x, y) on the z faces."""
        a = int(face) // 2
        return (self.ny, self.nx) if a == 2 else (self.nz, self.ny if a == 0 else self.nx)

    def set_inflow(self, face, state):
        """Boundary state of an INFLOW_EQ face: a per-height profile [nz, 3]
        (lbm_set_inflow) or one velocity per face cell [n2, n1, 3]
        (lbm_set_inflow_face, see face_shape)."""
        a = np.asarray(state, np.float64)
        if a.ndim == 3:
            arr = np.ascontiguousarray(a).reshape(self.face_shape(face) + (3,))
            self._check(self.lib.lbm_set_inflow_face(self.ctx, int(face), arr.ctypes.data_as(ctypes.c_void_p)))
            return
        prof = np.ascontiguousarray(a).reshape(self.nz, 3)
        self._check(self.lib.lbm_set_inflow(self.ctx, int(face), prof.ctypes.data_as(ctypes.c_void_p)))

    def halo_buffer(self):
        """Device buffer for one side's halo exchange: store [5][nz][nx]."""
        return torch.empty(5, self.nz, self.nx, dtype=self.store_dtype, device=self.device)

    def halo_pack(self, side, buf):
        """What this slab sends through side 0 (y-) or 1 (y+) after the last step."""
        self._check(self.lib.lbm_halo_pack(self.ctx, int(side), ctypes.c_void_p(buf.data_ptr())))

    def halo_unpack(self, side, buf):
        """Take what the neighbour on side 0 (y-) or 1 (y+) sent."""
        self._check(self.lib.lbm_halo_unpack(self.ctx, int(side), ctypes.c_void_p(buf.data_ptr())))

    def set_rotation(self, omega):
        """Rotation vector of the frame in lattice units (x, y, z); zero disables Coriolis."""
        om = np.ascontiguousarray(omega, np.float64).reshape(3)
        self._check(self.lib.lbm_set_rotation(self.ctx, om.ctypes.data_as(ctypes.c_void_p)))

    def set_turbulence(self, n_modes=64, length_scale=20.0, intensity=0.1, sigma0=0.0, gains=(1.0, 1.0, 1.0),
                       char_normal=False, inflow_only=False, shared=False, stride=1, interpolate=False,
                       seed=0, origin=(0.0, 0.0, 0.0), enable=True):
        """Synthetic von Karman inflow on the INFLOW_EQ faces (enable=False: off)."""
        if not enable:
            self._check(self.lib.lbm_set_turbulence(self.ctx, None))
            return
        t = _Turbulence()
        t.n_modes, t.stride, t.interpolate = int(n_modes), int(stride), int(bool(interpolate))
        t.char_normal, t.inflow_only, t.shared = int(bool(char_normal)), int(bool(inflow_only)), int(bool(shared))
        t.length_scale, t.intensity, t.sigma0 = float(length_scale), float(intensity), float(sigma0)
        for a in range(3):
            t.gain[a] = float(gains[a])
            t.origin[a] = float(origin[a])
        t.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        self._check(self.lib.lbm_set_turbulence(self.ctx, ctypes.byref(t)))

    def turbulence_info(self):
        n = ctypes.c_int64(0)
        u = ctypes.c_double(0.0)
        e = (ctypes.c_double * 3)()
        self._check(self.lib.lbm_turbulence_info(self.ctx, ctypes.byref(n), ctypes.byref(u), e))
        return int(n.value), float(u.value), np.array(list(e))

    def get_inflow(self, face):
        """Current boundary velocities of an INFLOW_EQ face, [n2, n1, 3] float64."""
        a = int(face) // 2
        shape = {0: (self.nz, self.ny), 1: (self.nz, self.nx), 2: (self.ny, self.nx)}[a]
        out = np.zeros(shape + (3,), np.float64)
        self._check(self.lib.lbm_get_inflow(self.ctx, int(face), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_sponge(self, width, strength):
        """Sponge / buffer nudging next to the INFLOW_EQ faces (width 0: off)."""
        self._check(self.lib.lbm_set_sponge(self.ctx, int(width), float(strength)))

    def balance_flux(self, mode):
        """Global flux balancing: 1 the boundary states now, 2 the full field every step, 0 off.
        Returns (phi_before, phi_after)."""
        a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(self.lib.lbm_balance_flux(self.ctx, int(mode), ctypes.byref(a), ctypes.byref(b)))
        return float(a.value), float(b.value)

    def net_flux(self):
        v = ctypes.c_double(0.0)
        self._check(self.lib.lbm_net_flux(self.ctx, ctypes.byref(v)))
        return float(v.value)

    def reset(self, u0=None):
        if u0 is None:
            self._check(self.lib.lbm_reset(self.ctx, None))
        else:
            u = np.ascontiguousarray(u0, np.float64)
            if u.ndim == 1:
                u = np.tile(u, (self.nz, 1))
            u = np.ascontiguousarray(u.reshape(self.nz, 3))
            self._check(self.lib.lbm_reset(self.ctx, u.ctypes.data_as(ctypes.c_void_p)))

    def step(self, n=1):
        self._check(self.lib.lbm_step(self.ctx, int(n)))

    def step_probed(self, n, acc):
        self._check(self.lib.lbm_step_probed(self.ctx, int(n), _ptr(acc)))

    @property
    def time(self):
        return int(self.lib.lbm_time(self.ctx))

    def cell_counts(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.lbm_cell_counts(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def layout(self):
        """(rows per block, rows per xy plane, x pitch) of the in-place array."""
        r, n, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.lbm_layout(self.ctx, ctypes.byref(r), ctypes.byref(n), ctypes.byref(p)))
        return r.value, n.value, p.value

    def macros(self):
        rho = torch.empty(self.nz, self.ny, self.nx, dtype=self.real_dtype, device=self.device)
        u = torch.empty(3, self.nz, self.ny, self.nx, dtype=self.real_dtype, device=self.device)
        nut = torch.empty_like(rho)
        self._check(self.lib.lbm_macros(self.ctx, _ptr(rho), _ptr(u), _ptr(nut)))
        return rho, u, nut

    def probe(self, pts):
        pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
        out = np.zeros((pts.shape[0], 4), np.float32)
        self._check(self.lib.lbm_probe(self.ctx, pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0],
                                       out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def probe_noalloc(self, pts):
        """lbm_probe through the library's fixed per-GPU scratch (no device allocation)."""
        pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
        out = np.zeros((pts.shape[0], 4), np.float32)
        self._check(self.lib.lbm_probe_noalloc(self.ctx, pts.ctypes.data_as(ctypes.c_void_p), pts.shape[0],
                                               out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def mass(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.lbm_mass(self.ctx, ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def new_state(self):
        return torch.empty(19, self.nz, self.ny, self.nx, dtype=self.store_dtype, device=self.device)

    def get_state(self, out=None):
        out = self.new_state() if out is None else out
        t = ctypes.c_int64()
        self._check(self.lib.lbm_get_state(self.ctx, _ptr(out), ctypes.byref(t)))
        return out, t.value

    def set_state(self, src, t):
        self._check(self.lib.lbm_set_state(self.ctx, _ptr(src), int(t)))

    def set_probes(self, cells):
        c = np.ascontiguousarray(cells, np.int32).reshape(-1, 3)
        self._check(self.lib.lbm_set_probes(self.ctx, c.ctypes.data_as(ctypes.c_void_p), c.shape[0]))
        self.np = c.shape[0]

    def probe_accumulate(self, acc):
        self._check(self.lib.lbm_probe_accumulate(self.ctx, _ptr(acc)))

    def set_stats(self, acc, stride):
        self._check(self.lib.lbm_set_stats(self.ctx, _ptr(acc), int(stride)))

    def push_step(self, src, dst):
        self._check(self.lib.lbm_push_step(self.ctx, _ptr(src), _ptr(dst)))

    def adjoint_step(self, f_t, lam_next, lam, probe_src=None, g_inflow=None):
        self._check(self.lib.lbm_adjoint_step(self.ctx, _ptr(f_t), _ptr(lam_next), _ptr(lam),
                                              _ptr(probe_src), _ptr(g_inflow)))

    def profile(self, enable=True):
        self._check(self.lib.lbm_profile(self.ctx, int(bool(enable))))

    def profile_read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.lbm_profile_read(self.ctx, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # -- conversions (host side, for comparisons) ----------------------------
    def state_to_f64(self, state):
        """Canonical stored state -> unshifted populations f (float64 numpy [19, nz, ny, nx])."""
        h = state.detach().to(torch.float64).cpu().numpy() / self.scale
        return h + (WEIGHTS * self.rho0)[:, None, None, None]

    def f64_to_state(self, f):
        h = (np.asarray(f, np.float64) - (WEIGHTS * self.rho0)[:, None, None, None]) * self.scale
        return torch.from_numpy(np.ascontiguousarray(h)).to(self.device).to(self.store_dtype)


def from_workload(w, storage=None, **kw):
    """GPU context for a workloads.Workload, inflow profiles set and state reset to its u0."""
    s = w.storage if storage is None else storage
    lat = LBM(w.nx, w.ny, w.nz, solid=w.solid, faces=w.faces, tau0=w.tau0, c_smag=w.c_smag,
              delta=w.delta, force=w.force, storage=s, noise_amp=w.noise_amp,
              noise_seed=w.noise_seed, **kw)
    for face, prof in w.inflow.items():
        lat.set_inflow(face, prof)
    if any(float(v) != 0.0 for v in w.omega):
        lat.set_rotation(w.omega)
    if w.sponge[0] > 0 and w.sponge[1] > 0.0:
        lat.set_sponge(*w.sponge)
    lat.reset(w.u0)
    return lat


def voxelize(shape, tris, starts, passes=1, solid=None):
    """Solid mask [nz, ny, nx] uint8: `solid` (or zeros) OR the voxelized
    closed meshes (tris [nt, 3, 3] lattice units, starts [nm + 1]) by the
    library's ray-parity kernels (lbm_voxelize)."""
    lib = load()
    nz, ny, nx = shape
    out = np.zeros(shape, np.uint8) if solid is None else np.array(solid, np.uint8, copy=True)
    out = np.ascontiguousarray(out)
    t = np.ascontiguousarray(tris, np.float64).reshape(-1, 9)
    s = np.ascontiguousarray(starts, np.int32)
    g = _Grid(nx, ny, nz)
    rc = lib.lbm_voxelize(ctypes.byref(g), t.ctypes.data_as(ctypes.c_void_p), int(t.shape[0]),
                          s.ctypes.data_as(ctypes.c_void_p), int(len(s) - 1), int(passes),
                          out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise LBMError(rc, lib.lbm_last_error(None).decode())
    return out


OMEGA_EARTH = 7.292115e-5   # rad/s, include/lbm.h LBM_OMEGA_EARTH (App. E)


def earth_rotation(latitude_deg: float, dt_si: float, grid_angle_deg: float = 0.0) -> np.ndarray:
    """lbm_earth_rotation: the Earth's rotation vector in lattice units in
    grid axes (App. E), for set_rotation."""
    lib = load()
    out = np.zeros(3, np.float64)
    rc = lib.lbm_earth_rotation(float(latitude_deg), float(dt_si), float(grid_angle_deg),
                                out.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise LBMError(rc, lib.lbm_last_error(None).decode())
    return out
