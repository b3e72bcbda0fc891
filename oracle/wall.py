"""Deformable B-spline wall in an inflow / outflow channel, the outflow-flux
losses, and the channel rollout with its adjoint (FP64 oracle; test
infrastructure only).

Paper, Sec. Projection: a solid enters the step only through its signed
distance phi (-> face fractions) and its velocity u_s; Sec. Back-propagation
through Geometry: dJ/dalpha and dJ/du_s are carried back through phi and u_s
to the shape parameters.  The channel configuration (readings, listed in the
design notes): a box [0, Lx] x [0, Ly] x [0, Lz], inflow on the z- side,
outflow (pressure 0) on the z+ side, walls elsewhere; the x- side carries a
deformable wall
    d(y, z, t) = amp * h(y, z) * s(t),   s(t) = (1 - cos(2 pi f t)) / 2,
    h(y, z) = sum_{m, n} a_{mn} B_m(y) B_n(z),
a uniform cubic B-spline with My x Mz control amplitudes a over [0, Ly] x
[0, Lz]: knot spacing D = L / (M - 3), control m centred at (m - 1) D, so the
M bases sum to one on the whole side and reproduce linear functions.  The
solid is x < d (phi = x - d > 0 is fluid) and moves along x with
dd/dt = amp * h * pi f sin(2 pi f t): only x faces carry a solid velocity.

Losses at each step n -> n+1, on the outlet faces (z faces on the z+ side):
the stored velocity is the face average alpha W + (1 - alpha) u_s (W the
fluid velocity, Eq. u_next_matrix), i.e. the flux density through the face,
so
    J_n = dt * dx^2 * sum_outlet w_f U^{n+1}_f,
with w = 1 (the total outflow flux) or a smooth window over the half x > Lx/2
of the outlet.

Pinned by: tests/test_oracle_wall.py (the cardinal cubic B-spline's values;
partition of unity and linear reproduction; a flat wall's exact fractions;
finite differences and the tangent / adjoint identity of the knot chain; the
total outflow flux equal to the geometry-only sum that the projection's
constraint implies, with its gradient: zero w.r.t. the velocity, the solid
flux's derivative w.r.t. the knots; finite differences of a windowed channel
rollout).
"""
from __future__ import annotations

import numpy as np

from .geometry import FaceGeometry, face_normal_axis
from .mac import Grid, WALL, INFLOW, OUTFLOW
from .projection import Operators
from .step import Step, StepParams

CHANNEL_BC = (WALL, WALL, WALL, WALL, INFLOW, OUTFLOW)


def bspline3(s):
    """Centred cardinal cubic B-spline (support [-2, 2])."""
    a = np.abs(np.asarray(s, float))
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3, np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def bspline_basis(s, M, L):
    """(N, M) values of the M uniform cubic B-spline bases over [0, L] at s."""
    D = L / (M - 3)
    return bspline3(np.asarray(s, float)[:, None] / D - (np.arange(M)[None, :] - 1.0))


def wall_time_factors(t, f):
    """s(t) = (1 - cos 2 pi f t) / 2 and ds/dt."""
    w = 2.0 * np.pi * f
    return 0.5 * (1.0 - np.cos(w * t)), np.pi * f * np.sin(w * t)


class WallGeometry(FaceGeometry):
    """Fractions and solid velocities of the B-spline wall at time t.

    ``vjp`` maps (dJ/dalpha, dJ/du_s) to dJ/da (My, Mz); ``jvp`` maps da to
    (dalpha, du_s).
    """

    def __init__(self, grid: Grid, knots, t, f, amp=0.1):
        self.knots = np.asarray(knots, float)
        My, Mz = self.knots.shape
        Ly, Lz = grid.n[1] * grid.dx, grid.n[2] * grid.dx
        self.s, self.sd = wall_time_factors(t, f)
        self.amp = float(amp)
        xn = grid.node_positions()
        self.By_n = bspline_basis(xn[:, 1], My, Ly)
        self.Bz_n = bspline_basis(xn[:, 2], Mz, Lz)
        h_n = np.einsum("nm,mk,nk->n", self.By_n, self.knots, self.Bz_n)
        phi = xn[:, 0] - self.amp * self.s * h_n
        # solid velocity: x faces only
        self.xf = face_normal_axis(grid) == 0
        xf_pos = grid.face_positions(0)
        self.By_f = bspline_basis(xf_pos[:, 1], My, Ly)
        self.Bz_f = bspline_basis(xf_pos[:, 2], Mz, Lz)
        h_f = np.einsum("nm,mk,nk->n", self.By_f, self.knots, self.Bz_f)
        us = np.zeros(grid.nfaces)
        us[self.xf] = self.amp * self.sd * h_f
        super().__init__(grid, phi, us)
        self.live_xf = ~self.fixed[self.xf]   # x faces whose u_s is not overridden by a domain side

    def vjp(self, galpha, gus):
        gphi = self.alpha_vjp(galpha)
        # phi = x - amp s h: d phi / d a_mn = -amp s By_m Bz_n
        ga = -self.amp * self.s * (self.By_n * gphi[:, None]).T @ self.Bz_n
        gx = np.where(self.live_xf, gus[self.xf], 0.0)
        ga += self.amp * self.sd * (self.By_f * gx[:, None]).T @ self.Bz_f
        return ga

    def jvp(self, da):
        da = np.asarray(da, float)
        dphi = -self.amp * self.s * np.sum((self.By_n @ da) * self.Bz_n, axis=1)
        dalpha = self.alpha_jvp(dphi)
        dus = np.zeros(self.grid.nfaces)
        dus[self.xf] = np.where(self.live_xf, self.amp * self.sd * np.sum((self.By_f @ da) * self.Bz_f, axis=1), 0.0)
        return dalpha, dus


# ---------------------------------------------------------------------------
# outflow-flux losses
# ---------------------------------------------------------------------------


def outlet_mask(grid: Grid):
    """Faces on the z+ side (the outlet)."""
    return grid.face_side() == 5


def outlet_window(grid: Grid, rng):
    """Smooth window over the half x > Lx/2 of the outlet (0 elsewhere):
    sin^2(2 pi (x/Lx - 1/2)) (1 + sin(2 pi y/Ly + psi) / 2), psi ~ U[0, 2 pi)."""
    psi = rng.uniform(0.0, 2.0 * np.pi)
    x = grid.all_face_positions()
    Lx, Ly = grid.n[0] * grid.dx, grid.n[1] * grid.dx
    xr = x[:, 0] / Lx
    w = np.where(xr > 0.5, np.sin(2.0 * np.pi * (xr - 0.5)) ** 2, 0.0) * (1.0 + 0.5 * np.sin(2.0 * np.pi * x[:, 1] / Ly + psi))
    return np.where(outlet_mask(grid), w, 0.0)


def flux_loss(grid: Grid, dt, u, w=None):
    """J = dt dx^2 sum_outlet w u (u: stored face-average velocity) and dJ/du."""
    m = outlet_mask(grid)
    wf = np.where(m, 1.0, 0.0) if w is None else np.asarray(w, float) * m
    c = dt * grid.dx * grid.dx
    return c * float(np.sum(wf * u)), c * wf


def constraint_net_orientation(grid: Grid, alpha):
    """D_f = sum over active cells c of G^T[c, f] (entries -1, 0, +1): the
    projection's constraint G^T U = 0 on every active cell sums to D . U = 0."""
    ops = Operators(grid, alpha)
    act = ops.active.astype(float)
    return np.asarray(ops.GT.T @ act).ravel()


# ---------------------------------------------------------------------------
# channel rollout
# ---------------------------------------------------------------------------


def channel_grid(n, dx, inflow=1.0):
    return Grid(n, dx, bc=CHANNEL_BC, inflow_speed=inflow)


class ChannelRollout:
    """Steps n -> n+1, n = 0 .. T-1, with the wall at t = (n + 1) dt, and the
    time-integrated outflow-flux loss sum_n J_n(U^{n+1})."""

    def __init__(self, prm: StepParams, u0, knots, f, steps, amp=0.1, window=None):
        self.prm = prm
        self.u0 = np.asarray(u0, float)
        self.knots = np.asarray(knots, float)
        self.f, self.T, self.amp = float(f), int(steps), float(amp)
        self.window = window

    def geometry(self, n):
        return WallGeometry(self.prm.grid, self.knots, (n + 1) * self.prm.dt, self.f, self.amp)

    def forward(self, keep=True):
        g, dt = self.prm.grid, self.prm.dt
        u = self.u0
        J = 0.0
        self.steps, self.geoms, self.hist = [], [], [u]
        for n in range(self.T):
            geo = self.geometry(n)
            st = Step(self.prm, u, geo.alpha, geo.us)
            u = st.result
            J += flux_loss(g, dt, u, self.window)[0]
            if keep:
                self.steps.append(st)
                self.geoms.append(geo)
            self.hist.append(u)
        self.J = J
        return J

    def backward(self):
        """(dJ/du0, dJ/da) of the time-integrated loss."""
        g, dt = self.prm.grid, self.prm.dt
        gu = np.zeros(g.nfaces)
        gk = np.zeros_like(self.knots)
        for n in range(self.T - 1, -1, -1):
            st, geo = self.steps[n], self.geoms[n]
            _, lu = flux_loss(g, dt, self.hist[n + 1], self.window)
            gu, g_alpha, g_us = st.vjp(gu + lu)
            gk += geo.vjp(g_alpha, g_us)
        return gu, gk
