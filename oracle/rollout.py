"""Rollouts, losses and back-propagation through time (FP64 oracle; test
infrastructure only).

Paper, Sec. Back-propagation through Time: the per-step adjoint is iterated
over the whole sequence in reverse; Sec. Back-propagation through Geometry:
dJ/dS and dJ/dU_s are carried back through the signed distance to the shape
parameters.

Rigid ellipsoid dynamics (a reading; the paper states only that controls act
on the parametric geometry): shape parameters theta0 = (c0, a, r0), with
R0 = Rodrigues(r0); per-step controls (v^n, w^n);
    c^{n+1} = c^n + dt v^n,    R^{n+1} = exp([dt w^n]_x) R^n,
and step n -> n+1 sees the solid at (c^{n+1}, a, R^{n+1}) moving with
u_s(x) = v^n + w^n x (x - c^{n+1}).

Losses: sum of u_f^2 over faces whose centre lies in the octant [0.5, 1]^3 of
the unit box, at the final step.

Pinned by: tests/test_oracle_rollout.py (central finite differences of the
loss w.r.t. shape parameters, controls and the initial velocity; Rodrigues
derivative against finite differences and orthogonality of R).
"""
from __future__ import annotations

import numpy as np

from .mac import Grid
from .geometry import EllipsoidGeometry, sphere_geometry, no_solid_geometry
from .step import Step, StepParams


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def rodrigues(r):
    """Rotation matrix exp([r]_x)."""
    t = np.linalg.norm(r)
    K = skew(r)
    if t == 0.0:
        return np.eye(3)
    return np.eye(3) + (np.sin(t) / t) * K + ((1.0 - np.cos(t)) / (t * t)) * (K @ K)


def rodrigues_grad(r):
    """dR/dr_i, (3, 3, 3) with [i] = dR/dr_i.

    Closed form of the derivative of the exponential map (Gallego & Yezzi,
    J. Math. Imaging Vis. 2015):
    dR/dr_i = (r_i [r]_x + [r x ((I - R) e_i)]_x) R / |r|^2, and [e_i]_x at r = 0.
    """
    t2 = float(r @ r)
    if t2 == 0.0:
        return np.stack([skew(e) for e in np.eye(3)])
    R = rodrigues(r)
    out = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        out.append((r[i] * skew(r) + skew(np.cross(r, (np.eye(3) - R) @ e))) @ R / t2)
    return np.stack(out)


def octant_mask(grid: Grid, lo=0.5):
    x = grid.all_face_positions()
    return np.all(x >= lo - 1e-12, axis=1)


def octant_loss(grid: Grid, u, lo=0.5):
    m = octant_mask(grid, lo)
    return float(np.sum(u[m] ** 2)), np.where(m, 2.0 * u, 0.0)


class EllipsoidRollout:
    """Forward rollout of the moving-ellipsoid scene and its full adjoint."""

    def __init__(self, prm: StepParams, u0, theta0, ctrl):
        self.prm = prm
        self.u0 = np.asarray(u0, float)
        self.theta0 = np.asarray(theta0, float)
        self.ctrl = np.asarray(ctrl, float)

    def poses(self):
        dt = self.prm.dt
        c = self.theta0[0:3].copy()
        R = rodrigues(self.theta0[6:9])
        out = []
        for n in range(self.ctrl.shape[0]):
            v, w = self.ctrl[n, :3], self.ctrl[n, 3:]
            c = c + dt * v
            R = rodrigues(dt * w) @ R
            out.append((c.copy(), R.copy()))
        return out

    def forward(self, keep=True):
        g = self.prm.grid
        a = self.theta0[3:6]
        u = self.u0
        self.steps, self.geoms, self.us_hist = [], [], [u]
        for n, (c, R) in enumerate(self.poses()):
            geo = EllipsoidGeometry(g, c, a, R, self.ctrl[n, :3], self.ctrl[n, 3:])
            st = Step(self.prm, u, geo.alpha, geo.us)
            u = st.result
            if keep:
                self.steps.append(st)
                self.geoms.append(geo)
            self.us_hist.append(u)
        return u

    def backward(self, gT):
        """Given dJ/du^T, return (dJ/du0, dJ/dtheta0 (9,), dJ/dctrl (T, 6))."""
        dt = self.prm.dt
        T = self.ctrl.shape[0]
        poses = self.poses()
        g = gT
        ga = np.zeros(3)
        gctrl = np.zeros_like(self.ctrl)
        gc_next = np.zeros(3)      # dJ/dc^{n+1} flowing back from later steps
        gR_next = np.zeros((3, 3))
        for n in range(T - 1, -1, -1):
            st, geo = self.steps[n], self.geoms[n]
            g, g_alpha, g_us = st.vjp(g)
            d = geo.vjp(g_alpha, g_us)
            gc = gc_next + d["c"]
            gR = gR_next + d["R"]
            ga += d["a"]
            gctrl[n, :3] += d["v"]
            gctrl[n, 3:] += d["w"]
            # c^{n+1} = c^n + dt v^n
            gctrl[n, :3] += dt * gc
            gc_next = gc
            # R^{n+1} = E R^n, E = exp([dt w^n]_x)
            Rn = poses[n - 1][1] if n > 0 else rodrigues(self.theta0[6:9])
            w = self.ctrl[n, 3:]
            E = rodrigues(dt * w)
            gE = gR @ Rn.T
            dE = rodrigues_grad(dt * w)
            gctrl[n, 3:] += dt * np.einsum("kij,ij->k", dE, gE)
            gR_next = E.T @ gR
        dR0 = rodrigues_grad(self.theta0[6:9])
        gr0 = np.einsum("kij,ij->k", dR0, gR_next)
        gtheta = np.concatenate([gc_next, ga, gr0])
        return g, gtheta, gctrl


class StaticRollout:
    """Forward rollout with a static solid (union of spheres, or none) and its adjoint
    w.r.t. the initial velocity."""

    def __init__(self, prm: StepParams, u0, spheres=None):
        self.prm = prm
        self.u0 = np.asarray(u0, float)
        g = prm.grid
        self.geo = sphere_geometry(g, spheres) if spheres is not None else no_solid_geometry(g)

    def forward(self, steps, keep=True):
        u = self.u0
        self.steps = []
        self.hist = [u]
        for _ in range(steps):
            st = Step(self.prm, u, self.geo.alpha, self.geo.us)
            u = st.result
            if keep:
                self.steps.append(st)
            self.hist.append(u)
        return u

    def backward(self, gT):
        g = gT
        for st in reversed(self.steps):
            g, _, _ = st.vjp(g)
        return g
