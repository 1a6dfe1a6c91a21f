"""Oracle of the open-boundary stabilisers (Sec. 2.2 and 2.3: mass-flux
consistency correction, global flux balancing, top sponge and lateral buffer
nudging).

TEST INFRASTRUCTURE ONLY: plain FP64 numpy; only tests/, the smoke check and
the benchmark's CPU baseline may use it.

Flux balancing.  Over the non-solid cells of the equilibrium-velocity faces
(INFLOW_EQ; a cell on two such faces belongs to the lower-numbered one) the
net outward volume flux is Phi = sum_i U_i . n_i (unit cell faces, n_i the
outward normal of the cell's face).  The smallest correction, in the
least-squares sense, of the normal velocities that makes Phi vanish is the
same shift for every cell, U_i -> U_i - (Phi / N) n_i.  Applied either to the
per-height profiles (every cell of a face row shares its profile entry) or
to the full per-cell boundary field.

Sponge and buffer nudging (readings: the paper names the layers and their
purpose but prints neither widths nor rates).  Next to every INFLOW_EQ face
other than the ground (x-, x+, y-, y+, z+), a cell at distance d = 1 .. W
from the face layer gets the strength s(d) = s_max ((W + 1 - d) / W)^2; a
cell near several faces takes the largest strength (the lower-numbered face
on ties).  After the collision the populations move toward the equilibrium
of the face's target velocity at the same density,
    f*_i += s (feq_i(rho, u_t) - feq_i(rho, u)),
with u the velocity of the collision and u_t the face's boundary state at
the cell's projection onto the face (a per-height profile: its value at the
cell's height, the top face's single row for the top sponge).  Mass is
unchanged and the momentum relaxes by s rho (u_t - u).
"""
from __future__ import annotations

import numpy as np

from . import INFLOW_EQ, equilibrium, face_value

NORMALS_OUT = -np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
SPONGE_FACES = (0, 1, 2, 3, 5)


def owner(faces, nx, ny, nz, x, y, z):
    on = (x == 0, x == nx - 1, y == 0, y == ny - 1, z == 0, z == nz - 1)
    for k in range(6):
        if on[k] and faces[k] == INFLOW_EQ:
            return k
    return -1


def boundary_cells(faces, solid):
    """[n, 4] rows (face, x, y, z) of non-solid cells on INFLOW_EQ faces."""
    nz, ny, nx = solid.shape
    rows = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid[z, y, x]:
                    continue
                f = owner(faces, nx, ny, nz, x, y, z)
                if f >= 0:
                    rows.append((f, x, y, z))
    return np.array(rows, np.int64).reshape(-1, 4)


def net_flux_field(faces, solid, field):
    """Phi over the boundary cells of a per-cell field [nz, ny, nx, 3]."""
    c = boundary_cells(faces, solid)
    u = field[c[:, 3], c[:, 2], c[:, 1]]
    return float(np.sum(np.einsum("na,na->n", u, NORMALS_OUT[c[:, 0]]))), len(c)


def balance_field(faces, solid, field):
    """Shift every boundary cell's normal velocity by -Phi/N; returns (field', Phi before, Phi after)."""
    phi, n = net_flux_field(faces, solid, field)
    out = np.array(field, np.float64, copy=True)
    if n == 0:
        return out, phi, phi
    c = boundary_cells(faces, solid)
    out[c[:, 3], c[:, 2], c[:, 1]] -= (phi / n) * NORMALS_OUT[c[:, 0]]
    return out, phi, net_flux_field(faces, solid, out)[0]


def net_flux_profiles(faces, solid, profiles):
    """Phi of the boundary states {face: [nz][3] profile or [n2][n1][3] per-cell array}."""
    c = boundary_cells(faces, solid)
    nz = solid.shape[0]
    u = np.array([face_value(profiles, f, x, y, z, nz) for f, x, y, z in c]).reshape(-1, 3)
    return float(np.sum(np.einsum("na,na->n", u, NORMALS_OUT[c[:, 0]]))), len(c)


def balance_profiles(faces, solid, profiles):
    """Same correction on the boundary states of the faces {face: [nz, 3]
    profile or [n2][n1][3] per-cell array}: every entry of a face moves by
    -(Phi / N) n_out."""
    phi, n = net_flux_profiles(faces, solid, profiles)
    out = {f: np.array(p, np.float64, copy=True) for f, p in profiles.items()}
    if n == 0:
        return out, phi, phi
    for f in out:
        out[f] -= (phi / n) * NORMALS_OUT[f][None, :]
    return out, phi, net_flux_profiles(faces, solid, out)[0]


def sponge_strength(faces, nx, ny, nz, width, s_max, x, y, z):
    """(strength, face) of the nudging at cell (x, y, z); (0, -1) outside the layers."""
    dist = (x, nx - 1 - x, y, ny - 1 - y, z, nz - 1 - z)
    best, face = 0.0, -1
    if width <= 0 or s_max <= 0.0:
        return best, face
    for f in SPONGE_FACES:
        if faces[f] != INFLOW_EQ:
            continue
        d = dist[f]
        if 1 <= d <= width:
            s = s_max * ((width + 1 - d) / width) ** 2
            if s > best:
                best, face = s, f
    return best, face


def nudge(fstar, rho, u, u_target, s):
    """f* + s (feq(rho, u_t) - feq(rho, u)) for one cell."""
    return fstar + s * (equilibrium(rho, u_target) - equilibrium(rho, u))


def target_velocity(profiles, face, nz, z, x=0, y=0):
    """Nudging target of `face` for the cell (x, y, z): the face's boundary
    state at the cell's projection onto the face."""
    return np.asarray(face_value(profiles, face, x, y, z, nz), np.float64)
