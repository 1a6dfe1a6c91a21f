"""Oracle of the synthetic von Karman inflow (App. F, turbulence generation).

TEST INFRASTRUCTURE ONLY: plain, slow FP64 numpy, written from the paper's
definitions in their order; only tests/, the smoke check and the benchmark's
CPU baseline may use it.

Steps (App. F):
  1. the active set: cells of the INFLOW_EQ faces x-, x+, y-, y+, z+ (the
     bottom face is left out, so is every solid cell), each cell on one face
     only (a cell on two inflow faces belongs to the lower-numbered one),
     optionally only cells whose mean velocity enters the domain,
     U_b . n_f > 0 with n_f the inward normal;
  2. per face the mean velocity and its characteristic speed |U_f| or
     |U_f . n_f|; faces at or below 1e-7 are dropped;
  3. over every remaining cell u_ref = mean |U_b| and e_c = sum U_b / |sum U_b|
     (fallback (1, 0, 0));
  4. per face (or one shared) realization of N_m modes: log-stratified k_m in
     [2 pi / (10 L), pi] (k_min = 0.1 k_max if the band is empty), isotropic
     direction, von Karman weight W(k) = k^4 / (1 + (k L)^2)^(17/6),
     amplitudes normalised to unit RMS per component, times the gains;
     omega_m = u_ref k_m . e_c; three independent phases per mode;
  5. q(x, t) = sum_m A_m cos(k_m . x - omega_m t + phi_m) with x the global
     lattice coordinates; sigma_i = I u_char (I > 0) else sigma_0;
     U_i(t) = U_b,i + sigma_i q(x_i, t);
  6. with a stride s, q is taken at anchors t_a = floor(t / s) s, held or
     interpolated linearly to t_a + s.

Readings (the paper leaves these open or states them two ways):
  * the phase is k . x - omega_m t: the text says the modes are convected
    along the mean-flow direction, which the printed "+ omega_m t" would
    reverse;
  * random numbers: uniform U = (splitmix64(seed + 2^32 (r + 1) + 6 m + j)
    >> 11) 2^-53 for realization r (the face index, or 0 when shared), mode
    m (from 0) and draw j: r_m (j = 0), mu = 2U - 1 (1), theta = 2 pi U (2),
    phi_x, phi_y, phi_z = 2 pi U (3, 4, 5);
  * one switch selects the norm |U| or the normal part |U . n| for both the
    face speed and u_char.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import INFLOW_EQ, face_value, splitmix64

NORMALS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
VK_FACES = (0, 1, 2, 3, 5)     # the bottom face (z-) is never perturbed


@dataclass
class VKParams:
    n_modes: int = 64
    length_scale: float = 20.0
    intensity: float = 0.1
    sigma0: float = 0.0
    gains: tuple = (1.0, 1.0, 1.0)
    char_normal: bool = False      # False: |U|, True: |U . n|
    inflow_only: bool = False
    shared: bool = False
    stride: int = 1
    interpolate: bool = False
    seed: int = 0
    origin: tuple = (0, 0, 0)      # global coordinates of cell (0, 0, 0)


def uniform(seed: int, r: int, m: int, j: int) -> float:
    return (splitmix64(seed + (r + 1) * 2 ** 32 + 6 * m + j) >> 11) * 2.0 ** -53


def owner_face(faces, nx, ny, nz, x, y, z):
    """Lowest-numbered INFLOW_EQ face the cell lies on, or -1."""
    on = (x == 0, x == nx - 1, y == 0, y == ny - 1, z == 0, z == nz - 1)
    for k in range(6):
        if on[k] and faces[k] == INFLOW_EQ:
            return k
    return -1


def active_cells(faces, solid, profiles, p: VKParams):
    """Step 1-3.  profiles: {face: [nz][3] per-height profile or [n2][n1][3]
    per-cell boundary state}, the mean boundary velocity U_b,i of each cell.
    Returns (cells [n, 4] = face, x, y, z; U_b [n, 3]; u_ref; e_c)."""
    nz, ny, nx = solid.shape
    rows = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid[z, y, x]:
                    continue
                f = owner_face(faces, nx, ny, nz, x, y, z)
                if f < 0 or f not in VK_FACES:
                    continue
                ub = np.asarray(face_value(profiles, f, x, y, z, nz), np.float64)
                if p.inflow_only and not ub @ NORMALS[f] > 0.0:
                    continue
                rows.append((f, x, y, z, ub))
    keep = []
    for f in VK_FACES:
        mine = [r for r in rows if r[0] == f]
        if not mine:
            continue
        mean = np.mean([r[4] for r in mine], axis=0)
        uc = abs(mean @ NORMALS[f]) if p.char_normal else np.linalg.norm(mean)
        if uc > 1e-7:
            keep += mine
    if not keep:
        return np.zeros((0, 4), np.int64), np.zeros((0, 3)), 0.0, np.array([1.0, 0.0, 0.0])
    cells = np.array([r[:4] for r in keep], np.int64)
    ub = np.array([r[4] for r in keep])
    u_ref = float(np.mean(np.linalg.norm(ub, axis=1)))
    s = ub.sum(axis=0)
    ns = np.linalg.norm(s)
    e_c = s / ns if ns > 0.0 else np.array([1.0, 0.0, 0.0])
    return cells, ub, u_ref, e_c


def mode_table(p: VKParams, r: int, u_ref: float, e_c):
    """Step 4 for realization r: wave vectors [N, 3], amplitudes [N, 3],
    frequencies [N], phases [N, 3]."""
    n = p.n_modes
    kmax = math.pi
    kmin = 2.0 * math.pi / (10.0 * p.length_scale)
    if not kmin < kmax:
        kmin = 0.1 * kmax
    k = np.zeros((n, 3))
    kmag = np.zeros(n)
    phi = np.zeros((n, 3))
    for m in range(n):
        u = [uniform(p.seed, r, m, j) for j in range(6)]
        xi = (m + u[0]) / n
        kmag[m] = math.exp(math.log(kmin) + xi * (math.log(kmax) - math.log(kmin)))
        mu = 2.0 * u[1] - 1.0
        th = 2.0 * math.pi * u[2]
        s = math.sqrt(1.0 - mu * mu)
        k[m] = kmag[m] * np.array([s * math.cos(th), s * math.sin(th), mu])
        phi[m] = [2.0 * math.pi * u[3], 2.0 * math.pi * u[4], 2.0 * math.pi * u[5]]
    W = kmag ** 4 / (1.0 + (kmag * p.length_scale) ** 2) ** (17.0 / 6.0)
    a = np.sqrt(W)
    A = a / math.sqrt(0.5 * np.sum(a * a))
    amp = A[:, None] * np.asarray(p.gains, np.float64)[None, :]
    omega = u_ref * (k @ np.asarray(e_c, np.float64))
    return k, amp, omega, phi, kmag


def q_series(k, amp, omega, phi, x, t):
    """q_alpha(x, t) = sum_m A_m,alpha cos(k_m . x - omega_m t + phi_m,alpha) at points x [n, 3]."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    base = x @ k.T - omega[None, :] * t                       # [n, N]
    out = np.zeros((x.shape[0], 3))
    for a in range(3):
        out[:, a] = np.sum(amp[None, :, a] * np.cos(base + phi[None, :, a]), axis=1)
    return out


class VonKarmanInflow:
    """The boundary velocity field U_i(t) of one grid, for the oracle."""

    def __init__(self, faces, solid, profiles, params: VKParams):
        self.p = params
        self.faces = list(faces)
        self.solid = np.asarray(solid)
        self.profiles = {k: np.asarray(v, np.float64) for k, v in profiles.items()}
        self.cells, self.ub, self.u_ref, self.e_c = active_cells(faces, self.solid, self.profiles, params)
        self.tables = {}
        for f in set(int(c) for c in self.cells[:, 0]):
            r = 0 if params.shared else f
            self.tables[f] = mode_table(params, r, self.u_ref, self.e_c)
        if params.intensity > 0.0:
            if params.char_normal:
                uc = np.abs(np.einsum("na,na->n", self.ub, NORMALS[self.cells[:, 0]]))
            else:
                uc = np.linalg.norm(self.ub, axis=1)
            self.sigma = params.intensity * uc
        else:
            self.sigma = np.full(len(self.cells), params.sigma0)
        self.xg = self.cells[:, 1:4].astype(np.float64) + np.asarray(params.origin, np.float64)[None, :]

    def q(self, t: float) -> np.ndarray:
        """q at every active cell at time t (no stride)."""
        out = np.zeros((len(self.cells), 3))
        for f, (k, amp, om, phi, _) in self.tables.items():
            sel = self.cells[:, 0] == f
            out[sel] = q_series(k, amp, om, phi, self.xg[sel], t)
        return out

    def q_strided(self, t: int) -> np.ndarray:
        s = self.p.stride
        if s <= 1:
            return self.q(t)
        ta = (t // s) * s
        if not self.p.interpolate:
            return self.q(ta)
        al = (t - ta) / s
        return (1.0 - al) * self.q(ta) + al * self.q(ta + s)

    def field(self, t: int) -> np.ndarray:
        """[nz, ny, nx, 3]: U_b at every inflow cell (its face's boundary
        state), U_b + sigma q at active ones."""
        nz, ny, nx = self.solid.shape
        out = np.zeros((nz, ny, nx, 3))
        for f, prof in self.profiles.items():
            if self.faces[f] != INFLOW_EQ:
                continue
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        if owner_face(self.faces, nx, ny, nz, x, y, z) == f:
                            out[z, y, x] = face_value(self.profiles, f, x, y, z, nz)
        if len(self.cells):
            v = self.ub + self.sigma[:, None] * self.q_strided(t)
            c = self.cells
            out[c[:, 3], c[:, 2], c[:, 1]] = v
        return out
