"""Semi-Lagrangian advection on the MAC grid, its tangent and its adjoint
(FP64 oracle; test infrastructure only).

Paper, Eq. advection_matrix: the advected field is a linear interpolation of
U^n at back-traced points, U~ = B(U^n) U^n.  App. B (Eqs. advection_1 and
advection_2) gives a two-stage (midpoint) time discretisation; read as an RK2
back-trace:

    v0    = V(u^n; x_f)
    x_mid = x_f - (dt/2) v0
    v1    = V(u^n; x_mid)
    x_src = x_f - dt v1
    U~_f  = I_d(u^n; x_src)

I_e is trilinear interpolation of component e on its own staggered lattice, in
index coordinates s_a = x_a/dx - o_a with o_a = 0 along e's own axis and 1/2
otherwise.  Each coordinate is clamped to [0, m_a - 1] (m_a lattice samples
along axis a) and the base index is min(floor(s), m_a - 2), so the floor cell
decides ties; along a periodic axis s wraps modulo n_a instead.  The
derivative of I_e w.r.t. position uses the same cell and is 0 along an axis
whose coordinate was clamped.  V = (I_x, I_y, I_z).

Viscosity (Eq. viscosity_matrix; App. B Eq. apply_force, explicit in time):
U^ = (I - nu dt / dx^2 G_f^T G_f) U~, where G_f is the difference operator of
each velocity component over the edges of its own face lattice (one row per
pair of neighbouring lattice points; edges wrap along periodic axes).  So
-G_f^T G_f is the per-component graph Laplacian: the 7-point Laplacian in the
interior, and no edge leaves the lattice at a domain side (the tangential
components see a zero normal derivative there, the normal component's
boundary faces are lattice points like any other).  A body force f (this
project's addition, used by the hydrostatic check) adds dt f on every face.

Pinned by: tests/test_oracle_advection.py (constant fields stay constant;
linear fields under uniform flow are translated exactly; an integer-cell shift
is exact; brute-force assembly of B at a tiny size; finite differences of the
tangent; the adjoint identity <J v, w> = <v, J^T w>).
"""
from __future__ import annotations

import numpy as np

from .mac import Grid


class Interp:
    """Trilinear interpolation set-up of component ``e`` at positions ``pos``."""

    def __init__(self, grid: Grid, e: int, pos: np.ndarray):
        self.grid, self.e = grid, e
        N = pos.shape[0]
        self.i0 = np.empty((N, 3), np.int64)
        self.i1 = np.empty((N, 3), np.int64)
        self.f = np.empty((N, 3))
        self.ds = np.empty((N, 3))          # d s_clamped / d x
        for a in range(3):
            off = 0.0 if a == e else 0.5
            s = pos[:, a] / grid.dx - off
            m = grid.m(e, a)
            if grid.periodic[a]:
                n = grid.n[a]
                s = np.mod(s, n)
                i0 = np.floor(s).astype(np.int64)
                i0 = np.minimum(i0, n - 1)
                f = s - i0
                i1 = (i0 + 1) % n
                ds = np.full(N, 1.0 / grid.dx)
            else:
                inside = (s >= 0.0) & (s <= m - 1)
                sc = np.clip(s, 0.0, m - 1)
                i0 = np.minimum(np.floor(sc).astype(np.int64), m - 2)
                f = sc - i0
                i1 = i0 + 1
                ds = np.where(inside, 1.0 / grid.dx, 0.0)
            self.i0[:, a], self.i1[:, a], self.f[:, a], self.ds[:, a] = i0, i1, f, ds
        self.shape = grid.face_shape(e)

    def _corners(self):
        """Yield (flat index, weight, dweight/dfrac (N,3)) for the 8 corners."""
        sz, sy, sx = self.shape
        for c in range(8):
            bits = [(c >> a) & 1 for a in range(3)]
            idx = [np.where(bits[a], self.i1[:, a], self.i0[:, a]) for a in range(3)]
            wa = [np.where(bits[a], self.f[:, a], 1.0 - self.f[:, a]) for a in range(3)]
            dwa = [np.full(self.f.shape[0], 1.0 if bits[a] else -1.0) for a in range(3)]
            flat = idx[0] + sx * (idx[1] + sy * idx[2])
            w = wa[0] * wa[1] * wa[2]
            dw = np.stack([dwa[0] * wa[1] * wa[2], wa[0] * dwa[1] * wa[2], wa[0] * wa[1] * dwa[2]], axis=1)
            yield flat, w, dw

    def value(self, comp_flat):
        out = np.zeros(self.f.shape[0])
        for flat, w, _ in self._corners():
            out += w * comp_flat[flat]
        return out

    def grad(self, comp_flat):
        """d value / d position, (N, 3)."""
        out = np.zeros((self.f.shape[0], 3))
        for flat, _, dw in self._corners():
            out += dw * comp_flat[flat][:, None]
        return out * self.ds

    def scatter(self, weights_per_point, size):
        """Transpose of ``value``: accumulate point weights into the lattice."""
        out = np.zeros(size)
        for flat, w, _ in self._corners():
            np.add.at(out, flat, w * weights_per_point)
        return out


def _components(grid, u):
    return [u[grid.face_offset(e):grid.face_offset(e) + grid.nf(e)] for e in range(3)]


class Advection:
    """One RK2 semi-Lagrangian advection of a face field, with tangent and adjoint."""

    def __init__(self, grid: Grid, u: np.ndarray, dt: float):
        self.grid, self.dt = grid, dt
        self.u = u
        uc = _components(grid, u)
        self.rec = []
        out = []
        for d in range(3):
            xf = grid.face_positions(d)
            I0 = [Interp(grid, e, xf) for e in range(3)]
            v0 = np.stack([I0[e].value(uc[e]) for e in range(3)], axis=1)
            xm = xf - 0.5 * dt * v0
            I1 = [Interp(grid, e, xm) for e in range(3)]
            v1 = np.stack([I1[e].value(uc[e]) for e in range(3)], axis=1)
            xs = xf - dt * v1
            I2 = Interp(grid, d, xs)
            out.append(I2.value(uc[d]))
            self.rec.append((I0, I1, I2))
        self.result = np.concatenate(out)

    def jvp(self, du):
        grid, dt = self.grid, self.dt
        uc = _components(grid, self.u)
        duc = _components(grid, du)
        out = []
        for d in range(3):
            I0, I1, I2 = self.rec[d]
            dv0 = np.stack([I0[e].value(duc[e]) for e in range(3)], axis=1)
            dxm = -0.5 * dt * dv0
            dv1 = np.stack([I1[e].value(duc[e]) + (I1[e].grad(uc[e]) * dxm).sum(axis=1)
                            for e in range(3)], axis=1)
            dxs = -dt * dv1
            out.append(I2.value(duc[d]) + (I2.grad(uc[d]) * dxs).sum(axis=1))
        return np.concatenate(out)

    def vjp(self, g):
        grid, dt = self.grid, self.dt
        uc = _components(grid, self.u)
        gc = [np.zeros(grid.nf(e)) for e in range(3)]
        gparts = _components(grid, g)
        for d in range(3):
            I0, I1, I2 = self.rec[d]
            gd = gparts[d]
            gc[d] += I2.scatter(gd, grid.nf(d))
            gxs = gd[:, None] * I2.grad(uc[d])
            gv1 = -dt * gxs
            gxm = np.zeros_like(gxs)
            for e in range(3):
                gc[e] += I1[e].scatter(gv1[:, e], grid.nf(e))
                gxm += gv1[:, e:e + 1] * I1[e].grad(uc[e])
            gv0 = -0.5 * dt * gxm
            for e in range(3):
                gc[e] += I0[e].scatter(gv0[:, e], grid.nf(e))
        return np.concatenate(gc)


def laplacian_periodic(grid: Grid, u):
    """Per-component 7-point Laplacian / dx^2 on fully periodic lattices."""
    if not all(grid.periodic):
        raise NotImplementedError("viscosity is defined here for periodic boxes only")
    out = []
    for e, comp in enumerate(grid.split(u)):
        lap = -6.0 * comp
        for ax in range(3):
            lap = lap + np.roll(comp, 1, axis=ax) + np.roll(comp, -1, axis=ax)
        out.append((lap / grid.dx ** 2).ravel())
    return np.concatenate(out)


def laplacian_faces(grid: Grid, u):
    """-G_f^T G_f u / dx^2: per component, the sum over the edges of its face
    lattice at each point of (neighbour - point) / dx^2 (edges wrap along
    periodic axes, and none leaves the lattice otherwise)."""
    out = []
    for e, comp in enumerate(grid.split(u)):
        lap = np.zeros_like(comp)
        for a in range(3):
            ax = 2 - a                      # numpy axis of grid axis a ([k][j][i] order)
            if grid.periodic[a]:
                lap = lap + (np.roll(comp, 1, axis=ax) - comp) + (np.roll(comp, -1, axis=ax) - comp)
            else:
                d = np.diff(comp, axis=ax)  # one value per edge
                lo = [slice(None)] * 3
                hi = [slice(None)] * 3
                lo[ax] = slice(0, -1)
                hi[ax] = slice(1, None)
                lap[tuple(lo)] += d         # the point below each edge gains (upper - lower)
                lap[tuple(hi)] -= d         # the point above it loses the same
        out.append((lap / grid.dx ** 2).ravel())
    return np.concatenate(out)


def body_force_faces(grid: Grid, f):
    return np.concatenate([np.full(grid.nf(d), float(f[d])) for d in range(3)])
