"""MAC grid and the discrete gradient G (FP64 oracle; test infrastructure only).

Sec. Numerical Simulation of the paper: pressure lives at cell centres,
velocity components on cell faces; (1/dx) G is the discrete gradient and
-(1/dx) G^T the discrete divergence.  Here G is assembled explicitly as a
sparse faces-by-cells matrix with entries +1 for the cell on the + side of a
face and -1 for the cell on its - side, so ``(G p)_f = p_{c+} - p_{c-}`` and
``(G^T v)_c = sum(lower faces of c) - sum(upper faces of c)``.

Domain sides carry one of the boundary kinds below.  A face on a non-periodic
domain side has only one cell, so its row of G has a single entry: that is
exactly a ghost pressure of 0 beyond the side, the Dirichlet condition
(App. B, Eq. bd:dirichlet) used on OUTFLOW sides.  On WALL / INFLOW sides the
face fraction is 0, so the ghost never enters the system (the Neumann
condition, Eq. bd:neumann, holds through the solid velocity).

Pinned by: tests/test_oracle_mac.py (G^T = -dx * divergence of closed-form
linear fields, G of a linear pressure = its exact face differences, row/column
structure at every boundary kind).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

WALL, INFLOW, OUTFLOW, PERIODIC = 0, 1, 2, 3


class Grid:
    """Uniform MAC grid of ``n = (nx, ny, nz)`` cells of width ``dx``.

    ``bc`` gives the kind of the six domain sides (x-, x+, y-, y+, z-, z+).
    Arrays use numpy shape ``[k][j][i]`` so that raveling puts x fastest.
    Along a periodic axis the face lattice of that axis' own component has
    ``n`` samples (face ``n`` is face ``0``); otherwise ``n + 1``.
    """

    def __init__(self, n, dx, bc=(WALL,) * 6, inflow_speed=0.0):
        self.n = tuple(int(v) for v in n)
        self.dx = float(dx)
        self.bc = tuple(int(b) for b in bc)
        self.inflow_speed = float(inflow_speed)
        self.periodic = []
        for a in range(3):
            lo, hi = self.bc[2 * a], self.bc[2 * a + 1]
            if (lo == PERIODIC) != (hi == PERIODIC):
                raise ValueError("periodic sides must come in pairs")
            self.periodic.append(lo == PERIODIC)

    # ---- sizes -------------------------------------------------------------
    def m(self, d, a):
        """Number of samples along axis ``a`` of the lattice of component ``d``."""
        if a == d and not self.periodic[a]:
            return self.n[a] + 1
        return self.n[a]

    def face_shape(self, d):
        return (self.m(d, 2), self.m(d, 1), self.m(d, 0))

    def nf(self, d):
        return int(np.prod(self.face_shape(d)))

    def face_offset(self, d):
        return sum(self.nf(e) for e in range(d))

    @property
    def nfaces(self):
        return self.face_offset(3)

    @property
    def cell_shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def ncells(self):
        return int(np.prod(self.n))

    @property
    def node_shape(self):
        return (self.n[2] + 1, self.n[1] + 1, self.n[0] + 1)

    def split(self, v):
        """Flat face vector -> list of the three component arrays (views)."""
        return [v[self.face_offset(d):self.face_offset(d) + self.nf(d)].reshape(self.face_shape(d))
                for d in range(3)]

    # ---- index helpers -----------------------------------------------------
    def face_ijk(self, d):
        """(i, j, k) integer arrays of every face of component ``d`` in flat order."""
        k, j, i = np.indices(self.face_shape(d))
        return i.ravel(), j.ravel(), k.ravel()

    def cell_flat(self, i, j, k):
        nx, ny, _ = self.n
        return i + nx * (j + ny * k)

    def face_positions(self, d):
        """(N, 3) physical positions of the faces of component ``d``."""
        ijk = self.face_ijk(d)
        pos = np.empty((ijk[0].size, 3))
        for a in range(3):
            off = 0.0 if a == d else 0.5
            pos[:, a] = (ijk[a] + off) * self.dx
        return pos

    def all_face_positions(self):
        return np.concatenate([self.face_positions(d) for d in range(3)], axis=0)

    def node_positions(self):
        k, j, i = np.indices(self.node_shape)
        return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) * self.dx

    def cell_positions(self):
        k, j, i = np.indices(self.cell_shape)
        return (np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) + 0.5) * self.dx

    def face_side(self):
        """Per face: -1 if interior (or periodic), else the domain side 0..5 it lies on."""
        out = []
        for d in range(3):
            own = self.face_ijk(d)[d]
            s = np.full(own.size, -1, dtype=np.int64)
            if not self.periodic[d]:
                s[own == 0] = 2 * d
                s[own == self.n[d]] = 2 * d + 1
            out.append(s)
        return np.concatenate(out)


def gradient_matrix(grid: Grid) -> sp.csr_matrix:
    """Sparse G (faces x cells): (G p)_f = p(cell on + side) - p(cell on - side)."""
    rows, cols, vals = [], [], []
    for d in range(3):
        i, j, k = grid.face_ijk(d)
        f = grid.face_offset(d) + np.arange(i.size)
        own = (i, j, k)[d]
        nd = grid.n[d]
        # + side cell: same index along d (exists unless this is the upper domain face)
        if grid.periodic[d]:
            plus_ok = np.ones(i.size, bool)
            plus_own = own % nd
            minus_ok = np.ones(i.size, bool)
            minus_own = (own - 1) % nd
        else:
            plus_ok = own < nd
            plus_own = own
            minus_ok = own >= 1
            minus_own = own - 1
        for ok, o, s in ((plus_ok, plus_own, 1.0), (minus_ok, minus_own, -1.0)):
            ci = [i, j, k]
            ci[d] = o
            c = grid.cell_flat(ci[0][ok], ci[1][ok], ci[2][ok])
            rows.append(f[ok])
            cols.append(c)
            vals.append(np.full(c.size, s))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.nfaces, grid.ncells))
