"""Slab decomposition along y with ghost rows and halo exchange (the domain
splitting behind the paper's multi-GPU runs), emulated in one process.

Every slab is an ordinary context whose interior y faces are LBM_HALO: its
first and/or last row is a ghost row standing for the neighbour's boundary
row.  After every step each slab packs the five crossing populations of
each interior side (lbm_halo_pack) and the neighbour unpacks them
(lbm_halo_unpack); with one process per GPU the buffers would travel by a
send/receive pair between neighbouring ranks instead of staying on one
device.  The slabs then reproduce the undecomposed run bit for bit.

Python here only slices the inputs, orders the calls and moves buffers;
every step and exchange runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding


def split_rows(ny: int, n: int):
    """[(y0, y1)] real-row ranges of n slabs covering [0, ny)."""
    edges = np.linspace(0, ny, n + 1).round().astype(int)
    if np.any(np.diff(edges) < 2):
        raise ValueError("every slab needs at least two real rows")
    return [(int(edges[k]), int(edges[k + 1])) for k in range(n)]


class SlabDecomposition:
    """n slabs of a workload (workloads.Workload), each with its own context."""

    def __init__(self, w, n: int, storage=None, rows=None):
        self.w = w
        self.n = int(n)
        self.rows = split_rows(w.ny, self.n) if rows is None else list(rows)
        self.slabs = []
        self.ghost = []        # (lower ghost, upper ghost) per slab, 0 or 1
        faces = [binding.FACE_KIND[f] if isinstance(f, str) else int(f) for f in w.faces]
        for k, (y0, y1) in enumerate(self.rows):
            lo, hi = int(k > 0), int(k < self.n - 1)
            a, b = y0 - lo, y1 + hi                       # rows of the slab, ghosts included
            fk = list(faces)
            if lo:
                fk[2] = binding.FACE_KIND["halo"]
            if hi:
                fk[3] = binding.FACE_KIND["halo"]
            lat = binding.LBM(w.nx, b - a, w.nz, solid=w.solid[:, a:b, :], faces=fk, tau0=w.tau0,
                              c_smag=w.c_smag, delta=w.delta, force=w.force,
                              storage=w.storage if storage is None else storage,
                              noise_amp=w.noise_amp, noise_seed=w.noise_seed)
            for face, state in w.inflow.items():
                if fk[face] != binding.FACE_KIND["inflow"]:
                    continue
                s = np.asarray(state, np.float64)
                if s.ndim == 3:                            # per-cell face states: take the slab's part
                    s = s[:, a:b, :] if face < 2 else (s[a:b] if face >= 4 else s)
                lat.set_inflow(face, s)
            if any(float(v) != 0.0 for v in w.omega):
                lat.set_rotation(w.omega)
            if w.sponge[0] > 0 and w.sponge[1] > 0.0:
                lat.set_sponge(*w.sponge)
            self.slabs.append(lat)
            self.ghost.append((lo, hi))
        self.bufs = [(s.halo_buffer() if lo else None, s.halo_buffer() if hi else None)
                     for s, (lo, hi) in zip(self.slabs, self.ghost)]

    def _span(self, k):
        (y0, y1), (lo, hi) = self.rows[k], self.ghost[k]
        return y0 - lo, y1 + hi

    def set_state(self, state: torch.Tensor, t: int = 0):
        """Scatter a canonical state of the whole grid [19][nz][ny][nx] (store
        type) into the slabs, ghost rows included."""
        for k, lat in enumerate(self.slabs):
            a, b = self._span(k)
            lat.set_state(state[:, :, a:b, :].contiguous(), t)

    def get_state(self) -> torch.Tensor:
        """The canonical state of the whole grid, from the slabs' real rows."""
        parts = []
        for k, lat in enumerate(self.slabs):
            s, _ = lat.get_state()
            lo, hi = self.ghost[k]
            parts.append(s[:, :, lo:s.shape[2] - hi, :])
        return torch.cat(parts, dim=2)

    def exchange(self):
        """The halo exchange after a step: every pack, then every unpack."""
        for k, lat in enumerate(self.slabs):
            lo_buf, hi_buf = self.bufs[k]
            if lo_buf is not None:
                lat.halo_pack(0, lo_buf)
            if hi_buf is not None:
                lat.halo_pack(1, hi_buf)
        for k, lat in enumerate(self.slabs):
            if self.ghost[k][0]:
                lat.halo_unpack(0, self.bufs[k - 1][1])   # what the slab below sent up
            if self.ghost[k][1]:
                lat.halo_unpack(1, self.bufs[k + 1][0])   # what the slab above sent down

    def step(self, n: int = 1):
        for _ in range(int(n)):
            for lat in self.slabs:
                lat.step(1)
            self.exchange()

    def close(self):
        for lat in self.slabs:
            lat.close()
