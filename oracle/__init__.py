"""Double-precision CPU oracle for the D3Q19 BGK + Smagorinsky update.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the HIP library
never does.  It wraps ``lbm_oracle.c`` (plain C loops, FP64, two lattices with
pull streaming) through ctypes and shares no code with the HIP path.

Arrays follow the oracle's own conventions: populations are unshifted ``f`` of
shape ``[19, nz, ny, nx]`` (float64), the solid mask is ``[nz, ny, nx]`` uint8,
inflow profiles are ``[6, nz, 3]`` float64 (face order x-, x+, y-, y+, z-, z+).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "lbm_oracle.c")]
# Builds of the same source: the plain one everything uses; "omp" splits the
# step's z planes over OpenMP threads (only to time the oracle on all host
# cores); "san" is instrumented with AddressSanitizer and UBSan (host code
# checks; load it in a process started with libasan preloaded).  The build a
# process loads is chosen by LBM_ORACLE_VARIANT ("", "omp" or "san").
_VARIANTS = {
    "": ([], "liboracle.so"),
    "omp": (["-fopenmp"], "liboracle_omp.so"),
    "san": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"],
            "liboracle_san.so"),
}
_LIB = os.path.join(_HERE, _VARIANTS[""][1])


def _lib_path(variant: str) -> str:
    return os.path.join(_HERE, _VARIANTS[variant][1])

PERIODIC, INFLOW_EQ, OUTFLOW_ZG, FREESLIP, WALL = 0, 1, 2, 3, 4
NQ = 19


def build(force: bool = True, variant: str = "") -> str:
    """Compile the oracle with gcc (strict IEEE: no contraction, no fast-math)."""
    flags, _ = _VARIANTS[variant]
    out = _lib_path(variant)
    if force or not os.path.exists(out):
        srcs = [s for s in _SRC if os.path.exists(s)]
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *flags, "-fPIC", "-shared",
               "-o", out + ".tmp", *srcs, "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


class _Cfg(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("face", ctypes.c_int32 * 6),
                ("tau0", ctypes.c_double), ("c_smag", ctypes.c_double),
                ("delta", ctypes.c_double), ("rho0", ctypes.c_double),
                ("force", ctypes.c_double * 3), ("omega", ctypes.c_double * 3),
                ("inflow_field", ctypes.c_void_p), ("sponge_strength", ctypes.c_double),
                ("sponge_width", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("face_base", ctypes.c_void_p * 6)]


_lib = None


def face_shape(face, nx, ny, nz):
    """(n2, n1) of a face's per-cell arrays: cell (j1, j2) of an x face is
    (y, z), of a y face (x, z), of a z face (x, y)."""
    a = face // 2
    return (ny, nx) if a == 2 else (nz, ny if a == 0 else nx)


def face_value(inflow, face, x, y, z, nz):
    """Boundary state of `face` at the face cell over (x, y, z) from
    {face: [nz][3] profile or [n2][n1][3] per-cell array}: the array entry
    of the cell's transverse coordinates, or the profile at its height (the
    top row for the z+ face)."""
    v = np.asarray(inflow[face], np.float64)
    if v.ndim == 3:
        a = face // 2
        return v[(y, x) if a == 2 else (z, y if a == 0 else x)]
    return v[nz - 1 if face == 5 else z]


def _load():
    global _lib
    if _lib is None:
        variant = os.environ.get("LBM_ORACLE_VARIANT", "")
        path = _lib_path(variant)
        if not os.path.exists(path):
            build(force=True, variant=variant)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.or_lattice.argtypes = [P, P, P]
        lib.or_equilibrium.argtypes = [ctypes.c_double, P, P]
        lib.or_moments.argtypes = [P, P, P, P]
        lib.or_tau_eff.argtypes = [ctypes.c_double] * 5
        lib.or_tau_eff.restype = ctypes.c_double
        lib.or_q_invariant.argtypes = [P, P, P]
        lib.or_q_invariant.restype = ctypes.c_double
        lib.or_collide.argtypes = [P, P, P, P, P]
        lib.or_collide.restype = ctypes.c_double
        lib.or_splitmix64.argtypes = [ctypes.c_uint64]
        lib.or_splitmix64.restype = ctypes.c_uint64
        lib.or_init.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_uint64, P]
        lib.or_step.argtypes = [P, P, P, P, P, P]
        lib.or_run.argtypes = [P, P, P, P, ctypes.c_int64]
        lib.or_macros.argtypes = [P, P, P, P, P, P, P]
        lib.or_mass.argtypes = [P, P, P, P, P]
        lib.or_last_error.restype = ctypes.c_int
        lib.or_collide_jacobian.argtypes = [P, P, P]
        lib.or_adjoint_step.argtypes = [P, P, P, P, P, P, P, ctypes.c_int32, P, P, P]
        lib.or_adjoint_step.restype = ctypes.c_int
        lib.or_step_cell.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.or_collide_cell.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.or_step_cell.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def lattice():
    """(c [19,3] int, w [19] float64, opp [19] int) as the oracle defines them."""
    lib = _load()
    c = np.zeros((NQ, 3), np.int32)
    w = np.zeros(NQ, np.float64)
    opp = np.zeros(NQ, np.int32)
    lib.or_lattice(_p(c), _p(w), _p(opp))
    return c, w, opp


def equilibrium(rho: float, u) -> np.ndarray:
    lib = _load()
    u = np.ascontiguousarray(u, np.float64)
    out = np.zeros(NQ, np.float64)
    lib.or_equilibrium(float(rho), _p(u), _p(out))
    return out


def tau_eff(tau0, c_smag, delta, q, rho) -> float:
    return _load().or_tau_eff(tau0, c_smag, delta, q, rho)


def splitmix64(x: int) -> int:
    return int(_load().or_splitmix64(x & 0xFFFFFFFFFFFFFFFF))


class Oracle:
    """One configured oracle lattice (geometry, faces, collision parameters)."""

    def __init__(self, nx, ny, nz, faces, tau0, c_smag=0.0, delta=1.0, rho0=1.0,
                 force=(0.0, 0.0, 0.0), solid=None, inflow=None, omega=(0.0, 0.0, 0.0), sponge=(0, 0.0)):
        self.shape = (nz, ny, nx)
        self.cfg = _Cfg()
        self.cfg.nx, self.cfg.ny, self.cfg.nz = nx, ny, nz
        for k in range(6):
            self.cfg.face[k] = int(faces[k])
        self.cfg.tau0, self.cfg.c_smag, self.cfg.delta, self.cfg.rho0 = tau0, c_smag, delta, rho0
        for a in range(3):
            self.cfg.force[a] = float(force[a])
            self.cfg.omega[a] = float(omega[a])
        self.cfg.sponge_width, self.cfg.sponge_strength = int(sponge[0]), float(sponge[1])
        self.solid = np.zeros(self.shape, np.uint8) if solid is None else \
            np.ascontiguousarray(solid, np.uint8).reshape(self.shape)
        self.inflow = np.zeros((6, nz, 3), np.float64)
        self._face_base = {}
        if inflow is not None:
            for face, prof in inflow.items():
                a = np.asarray(prof, np.float64)
                if a.ndim == 3:   # per-cell boundary state of the face, [n2][n1][3]
                    a = np.ascontiguousarray(a).reshape(face_shape(face, nx, ny, nz) + (3,))
                    self._face_base[face] = a
                    self.cfg.face_base[face] = a.ctypes.data
                else:
                    self.inflow[face] = a.reshape(nz, 3)
        self.lib = _load()
        self._field = None

    @property
    def inflow_field(self):
        """Optional velocity of every inflow cell, [nz, ny, nx, 3] (None: the
        per-height profiles).  Read only at inflow cells."""
        return self._field

    @inflow_field.setter
    def inflow_field(self, v):
        if v is None:
            self._field = None
            self.cfg.inflow_field = None
            return
        a = np.ascontiguousarray(v, np.float64).reshape(self.shape + (3,))
        self._field = a
        self.cfg.inflow_field = a.ctypes.data

    @property
    def n(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}")

    def init(self, u0=None, amp=0.0, seed=0) -> np.ndarray:
        nz = self.shape[0]
        u0 = np.zeros((nz, 3)) if u0 is None else np.asarray(u0, np.float64)
        if u0.ndim == 1:
            u0 = np.tile(u0, (nz, 1))
        u0 = np.ascontiguousarray(u0, np.float64)
        f = np.zeros((NQ,) + self.shape, np.float64)
        self._check(self.lib.or_init(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow), _p(u0),
                                     float(amp), int(seed), _p(f)))
        return f

    def step(self, f: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(f, np.float64)
        out = np.empty_like(f)
        work = np.empty_like(f)
        self._check(self.lib.or_step(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow), _p(f),
                                     _p(out), _p(work)))
        return out

    def run(self, f: np.ndarray, steps: int) -> np.ndarray:
        f = np.array(f, np.float64, order="C", copy=True)
        self._check(self.lib.or_run(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow), _p(f),
                                    int(steps)))
        return f

    def macros(self, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        nut = np.zeros(self.shape)
        self.lib.or_macros(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow), _p(f), _p(rho),
                           _p(u), _p(nut))
        return rho, u, nut

    def mass(self, f: np.ndarray):
        f = np.ascontiguousarray(f, np.float64)
        m = np.zeros(1)
        e = np.zeros(1)
        self.lib.or_mass(ctypes.byref(self.cfg), _p(self.solid), _p(f), _p(m), _p(e))
        return float(m[0]), float(e[0])

    def collide(self, fcell):
        """Collide one cell: returns (f*, rho, u, tau_eff)."""
        fcell = np.ascontiguousarray(fcell, np.float64)
        out = np.zeros(NQ)
        rho = np.zeros(1)
        u = np.zeros(3)
        tau = self.lib.or_collide(ctypes.byref(self.cfg), _p(fcell), _p(out), _p(rho), _p(u))
        return out, float(rho[0]), u, tau

    def collide_cell(self, fcell, x, y, z):
        """Post-collision populations of one interior cell at (x, y, z),
        including the sponge / buffer nudging there."""
        fcell = np.ascontiguousarray(fcell, np.float64)
        out = np.zeros(NQ)
        self.lib.or_collide_cell(ctypes.byref(self.cfg), _p(self.inflow), _p(fcell), int(x), int(y), int(z),
                                 _p(out))
        return out

    def moments(self, fcell):
        fcell = np.ascontiguousarray(fcell, np.float64)
        rho = np.zeros(1)
        u = np.zeros(3)
        self.lib.or_moments(ctypes.byref(self.cfg), _p(fcell), _p(rho), _p(u))
        return float(rho[0]), u

    def q_invariant(self, fcell, feq):
        pi = np.zeros(9)
        q = self.lib.or_q_invariant(_p(np.ascontiguousarray(fcell, np.float64)),
                                    _p(np.ascontiguousarray(feq, np.float64)), _p(pi))
        return q, pi.reshape(3, 3)

    def collide_jacobian(self, fcell):
        """J[i, j] = d f*_i / d f_j of the collision of one cell."""
        J = np.zeros((NQ, NQ))
        self.lib.or_collide_jacobian(ctypes.byref(self.cfg), _p(np.ascontiguousarray(fcell, np.float64)), _p(J))
        return J

    def adjoint_step(self, f_t, lam_next, probes=None, probe_src=None):
        """lam(t) = (d f(t+1)/d f(t))^T lam_next + probe sources at time t, and
        the gradient of the step with respect to the inflow profiles [6, nz, 3]."""
        f_t = np.ascontiguousarray(f_t, np.float64)
        lam_next = np.ascontiguousarray(lam_next, np.float64)
        lam = np.zeros_like(f_t)
        work = np.zeros_like(f_t)
        g = np.zeros((6, self.shape[0], 3))
        if probes is None:
            pr, np_, src = None, 0, None
        else:
            pr = np.ascontiguousarray(probes, np.int32).reshape(-1, 3)
            np_ = pr.shape[0]
            src = None if probe_src is None else np.ascontiguousarray(probe_src, np.float64).reshape(-1, 3)
        self._check(self.lib.or_adjoint_step(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow), _p(f_t),
                                             _p(lam_next), _p(lam), None if pr is None else _p(pr), np_,
                                             None if src is None else _p(src), _p(g), _p(work)))
        return lam, g

    def step_cell(self, window, x, y, z):
        """f(x, t+1) of one cell from the 5x5x5 window of f(t) around it."""
        out = np.zeros(NQ)
        self._check(self.lib.or_step_cell(ctypes.byref(self.cfg), _p(self.solid), _p(self.inflow),
                                          _p(np.ascontiguousarray(window, np.float64)), x, y, z, _p(out)))
        return out
