"""One operator-split step n -> n+1 with its tangent and adjoint (FP64 oracle;
test infrastructure only).

Paper, Sec. Numerical Simulation: advection (Eq. advection_matrix), viscosity
(Eq. viscosity_matrix; App. B Eq. apply_force), an optional body force (this
project's addition, for the hydrostatic check),
projection (Eqs. projection_matrix, u_next_matrix).  Back-propagation mirrors
the forward in reverse order (Sec. Back-propagation through Time): projection
first, then viscosity and advection.  The geometry enters only through the
face fractions alpha and the solid face velocity u_s (Sec. Back-propagation
through Geometry); this module returns dJ/dalpha and dJ/du_s and leaves the
chain to the shape parameters to ``geometry`` / ``rollout``.

Pinned by: tests/test_oracle_step.py (rest stays at rest; hydrostatic
balance; Taylor-Green decay in a periodic box with first-order convergence;
the adjoint identity <J v, w> = <v, J^T w> against the tangent; an independent
PyTorch float64 brute-force forward with a dense solve, differentiated by
autograd, at a tiny size; central finite differences).
"""
from __future__ import annotations

import numpy as np

from .mac import Grid
from .advection import Advection, laplacian_faces, body_force_faces
from .projection import Projection


class StepParams:
    def __init__(self, grid: Grid, dt, rho=1.0, nu=0.0, gravity=(0.0, 0.0, 0.0), tol=1e-12,
                 method="pcg"):
        self.grid, self.dt, self.rho, self.nu = grid, float(dt), float(rho), float(nu)
        self.gravity = np.asarray(gravity, float)
        self.tol, self.method = tol, method

    @property
    def k(self):
        return self.dt / (self.rho * self.grid.dx)


class Step:
    """Forward of one step; keeps what the tangent and adjoint need."""

    def __init__(self, prm: StepParams, u, alpha, us):
        self.prm = prm
        g = prm.grid
        self.adv = Advection(g, u, prm.dt)
        ut = self.adv.result
        if prm.nu != 0.0:
            ut = ut + prm.dt * prm.nu * laplacian_faces(g, ut)
        if np.any(prm.gravity != 0.0):
            ut = ut + prm.dt * body_force_faces(g, prm.gravity)
        self.uhat = ut
        self.proj = Projection(g, ut, alpha, us, prm.k, prm.tol, prm.method)
        self.result = self.proj.result
        self.P = self.proj.P

    def jvp(self, du, dalpha, dus):
        prm = self.prm
        d = self.adv.jvp(du)
        if prm.nu != 0.0:
            d = d + prm.dt * prm.nu * laplacian_faces(prm.grid, d)
        return self.proj.jvp(d, dalpha, dus)

    def vjp(self, g):
        """dJ/dU^{n+1} -> (dJ/dU^n, dJ/dalpha, dJ/du_s)."""
        prm = self.prm
        g_uhat, g_alpha, g_us = self.proj.vjp(g)
        if prm.nu != 0.0:       # -G_f^T G_f is symmetric
            g_uhat = g_uhat + prm.dt * prm.nu * laplacian_faces(prm.grid, g_uhat)
        return self.adv.vjp(g_uhat), g_alpha, g_us
