"""Solid geometry -> face fluid fractions and solid face velocities (FP64 oracle;
test infrastructure only).

Paper, Sec. Projection (cut-cell paragraph): the solid's signed distance phi and
velocity u_s come from the geometry; the zero contour of phi is intersected with
each grid face, and alpha_f is the fluid share of the face's area.  The paper
prints the case with one fluid corner A (neighbours B, D solid):
alpha = 1/2 * phi_A/(phi_A - phi_B) * phi_A/(phi_A - phi_D).
Readings used here (listed in the design notes):

* phi > 0 is fluid, phi <= 0 solid (the printed triangle is the fluid part);
* every other corner configuration follows the same linear edge interpolation
  (2D marching squares): 3 fluid corners -> 1 - the solid corner's triangle;
  2 adjacent -> trapezoid; 2 diagonal (saddle) -> decided by the sign of the
  corner mean (positive: fluid connects, 1 - two solid triangles);
* corners of an x-face (i,j,k) are the nodes (i,j,k), (i,j+1,k), (i,j+1,k+1),
  (i,j,k+1) in cyclic order (y- and z-faces alike);
* u_s at a face is the normal component of the solid velocity at the face centre.

Solids: union of spheres (phi = min_i |x - c_i| - r_i, static); rigid ellipsoid
with centre c, semi-axes a and rotation R (body -> world), using the distance
estimate phi = k0 (k0 - 1) / k1 with p = R^T (x - c), k0 = |p / a|,
k1 = |p / a^2| (exact zero set; equals |x - c| - r for a sphere), moving with
u_s(x) = v + w x (x - c).

Pinned by: tests/test_oracle_geometry.py (the printed triangle value; exact
areas for planar phi in every non-saddle case; complement symmetry; all-fluid /
all-solid; the ellipsoid reducing to the sphere distance; finite differences of
every derivative here).
"""
from __future__ import annotations

import numpy as np

from .mac import Grid, WALL, INFLOW, OUTFLOW, PERIODIC

# ---------------------------------------------------------------------------
# signed distances
# ---------------------------------------------------------------------------


def phi_spheres(x, spheres):
    """Union of spheres: min over spheres of |x - c| - r.  x: (N, 3)."""
    sph = np.atleast_2d(spheres)
    d = np.linalg.norm(x[:, None, :] - sph[None, :, :3], axis=2) - sph[None, :, 3]
    return d.min(axis=1)


def phi_ellipsoid(x, c, a, R, with_grad=False):
    """Ellipsoid distance estimate and (optionally) its partials w.r.t. c, a, R.

    Returns phi (N,), and if ``with_grad``: dphi/dc (N,3), dphi/da (N,3),
    dphi/dR (N,3,3).
    """
    r = x - c[None, :]
    p = r @ R                       # p_j = sum_i r_i R_ij  (= R^T r)
    q = p / a[None, :]
    s = p / (a * a)[None, :]
    k0 = np.linalg.norm(q, axis=1)
    k1 = np.linalg.norm(s, axis=1)
    centre = k1 == 0.0
    k1s = np.where(centre, 1.0, k1)
    k0s = np.where(centre, 1.0, k0)
    phi = np.where(centre, -a.min(), k0 * (k0 - 1.0) / k1s)
    if not with_grad:
        return phi
    dphi_dk0 = (2.0 * k0 - 1.0) / k1s
    dphi_dk1 = -k0 * (k0 - 1.0) / (k1s * k1s)
    dk0_dp = q / (k0s[:, None] * a[None, :])
    dk1_dp = s / (k1s[:, None] * (a * a)[None, :])
    g = dphi_dk0[:, None] * dk0_dp + dphi_dk1[:, None] * dk1_dp      # dphi/dp
    dk0_da = -(q * q) / (k0s[:, None] * a[None, :])
    dk1_da = -2.0 * (s * s) / (k1s[:, None] * a[None, :])
    ga = dphi_dk0[:, None] * dk0_da + dphi_dk1[:, None] * dk1_da
    gc = -(g @ R.T)                                                  # -sum_j g_j R_ij
    gR = r[:, :, None] * g[:, None, :]                               # r_i g_j
    z = centre[:, None]
    return phi, np.where(z, 0.0, gc), np.where(z, 0.0, ga), np.where(centre[:, None, None], 0.0, gR)


# ---------------------------------------------------------------------------
# marching squares on one face
# ---------------------------------------------------------------------------


def _t(a, b):
    """Fraction along an edge from the corner with value a to the sign change."""
    return a / (a - b)


def _dt(a, b):
    den = (a - b) ** 2
    return -b / den, a / den


def face_fraction(phis):
    """Fluid area fraction of faces from their 4 cyclic corner values.

    phis: (N, 4).  Returns alpha (N,) and dalpha/dphi (N, 4).
    """
    phis = np.asarray(phis, dtype=np.float64)
    N = phis.shape[0]
    fluid = phis > 0.0
    cnt = fluid.sum(axis=1)
    alpha = np.zeros(N)
    grad = np.zeros((N, 4))
    alpha[cnt == 4] = 1.0
    mean = phis.mean(axis=1)
    for k in range(4):
        idx = (np.arange(4) + k) % 4          # rolled corner order: k, k+1, k+2, k+3
        P = phis[:, idx]
        F = fluid[:, idx]
        G = np.zeros((N, 4))                  # gradient in rolled order
        # one fluid corner at position k
        m1 = (cnt == 1) & F[:, 0]
        if m1.any():
            a, b, d = P[m1, 0], P[m1, 1], P[m1, 3]
            tb, td = _t(a, b), _t(a, d)
            alpha[m1] = 0.5 * tb * td
            ta_b, tb_b = _dt(a, b)
            ta_d, td_d = _dt(a, d)
            Gm = np.zeros((m1.sum(), 4))
            Gm[:, 0] = 0.5 * (ta_b * td + tb * ta_d)
            Gm[:, 1] = 0.5 * tb_b * td
            Gm[:, 3] = 0.5 * tb * td_d
            G[m1] = Gm
        # one solid corner at position k
        m3 = (cnt == 3) & ~F[:, 0]
        if m3.any():
            a, b, d = P[m3, 0], P[m3, 1], P[m3, 3]
            tb, td = _t(a, b), _t(a, d)
            alpha[m3] = 1.0 - 0.5 * tb * td
            ta_b, tb_b = _dt(a, b)
            ta_d, td_d = _dt(a, d)
            Gm = np.zeros((m3.sum(), 4))
            Gm[:, 0] = -0.5 * (ta_b * td + tb * ta_d)
            Gm[:, 1] = -0.5 * tb_b * td
            Gm[:, 3] = -0.5 * tb * td_d
            G[m3] = Gm
        # two adjacent fluid corners at positions k, k+1
        m2 = (cnt == 2) & F[:, 0] & F[:, 1]
        if m2.any():
            a0, a1, a2, a3 = P[m2, 0], P[m2, 1], P[m2, 2], P[m2, 3]
            t03, t12 = _t(a0, a3), _t(a1, a2)
            alpha[m2] = 0.5 * (t03 + t12)
            d0, d3 = _dt(a0, a3)
            d1, d2 = _dt(a1, a2)
            Gm = np.zeros((m2.sum(), 4))
            Gm[:, 0] = 0.5 * d0
            Gm[:, 3] = 0.5 * d3
            Gm[:, 1] = 0.5 * d1
            Gm[:, 2] = 0.5 * d2
            G[m2] = Gm
        # two diagonal fluid corners at positions k, k+2 (each pair seen twice: k < 2 only)
        if k < 2:
            md = (cnt == 2) & F[:, 0] & F[:, 2]
            if md.any():
                a0, a1, a2, a3 = P[md, 0], P[md, 1], P[md, 2], P[md, 3]
                Gm = np.zeros((md.sum(), 4))
                conn = mean[md] > 0.0
                # connected fluid: 1 - solid triangles at corners 1 and 3
                s10, s12 = _t(a1, a0), _t(a1, a2)
                s30, s32 = _t(a3, a0), _t(a3, a2)
                # separate fluid: triangles at corners 0 and 2
                f01, f03 = _t(a0, a1), _t(a0, a3)
                f21, f23 = _t(a2, a1), _t(a2, a3)
                alpha[md] = np.where(conn, 1.0 - 0.5 * s10 * s12 - 0.5 * s30 * s32,
                                     0.5 * f01 * f03 + 0.5 * f21 * f23)
                # connected-case gradient
                d1a, d0a = _dt(a1, a0)
                d1b, d2b = _dt(a1, a2)
                d3a, d0c = _dt(a3, a0)
                d3b, d2c = _dt(a3, a2)
                gc = np.zeros((md.sum(), 4))
                gc[:, 1] = -0.5 * (d1a * s12 + s10 * d1b)
                gc[:, 3] = -0.5 * (d3a * s32 + s30 * d3b)
                gc[:, 0] = -0.5 * (d0a * s12) - 0.5 * (d0c * s32)
                gc[:, 2] = -0.5 * (s10 * d2b) - 0.5 * (s30 * d2c)
                # separate-case gradient
                e0a, e1a = _dt(a0, a1)
                e0b, e3b = _dt(a0, a3)
                e2a, e1b = _dt(a2, a1)
                e2b, e3c = _dt(a2, a3)
                gs = np.zeros((md.sum(), 4))
                gs[:, 0] = 0.5 * (e0a * f03 + f01 * e0b)
                gs[:, 2] = 0.5 * (e2a * f23 + f21 * e2b)
                gs[:, 1] = 0.5 * (e1a * f03 + f23 * e1b)
                gs[:, 3] = 0.5 * (f01 * e3b + f21 * e3c)
                Gm = np.where(conn[:, None], gc, gs)
                G[md] = Gm
        # un-roll: rolled position r is corner (r + k) % 4
        grad[:, idx] += G
    return alpha, grad


def face_corner_nodes(grid: Grid):
    """(F, 4) flat node indices of the cyclic corners of every face (canonical order)."""
    nx, ny, _ = grid.n
    sx, sy = nx + 1, ny + 1

    def nid(i, j, k):
        return i + sx * (j + sy * k)

    out = []
    for d in range(3):
        i, j, k = grid.face_ijk(d)
        if d == 0:
            c = [nid(i, j, k), nid(i, j + 1, k), nid(i, j + 1, k + 1), nid(i, j, k + 1)]
        elif d == 1:
            c = [nid(i, j, k), nid(i + 1, j, k), nid(i + 1, j, k + 1), nid(i, j, k + 1)]
        else:
            c = [nid(i, j, k), nid(i + 1, j, k), nid(i + 1, j + 1, k), nid(i, j + 1, k)]
        out.append(np.stack(c, axis=1))
    return np.concatenate(out, axis=0)


# ---------------------------------------------------------------------------
# solid velocity and domain boundary overrides
# ---------------------------------------------------------------------------


def face_normal_axis(grid: Grid):
    return np.concatenate([np.full(grid.nf(d), d) for d in range(3)])


def rigid_face_velocity(grid: Grid, c, v, w):
    """Normal component of u_s(x) = v + w x (x - c) at every face centre."""
    x = grid.all_face_positions()
    r = x - c[None, :]
    vel = v[None, :] + np.cross(w[None, :], r)
    ax = face_normal_axis(grid)
    return vel[np.arange(ax.size), ax]


def rigid_face_velocity_partials(grid: Grid, c, v, w):
    """d u_s,f / d(v, w, c) for every face: (F, 3) each."""
    x = grid.all_face_positions()
    r = x - c[None, :]
    ax = face_normal_axis(grid)
    F = ax.size
    dv = np.zeros((F, 3))
    dv[np.arange(F), ax] = 1.0
    # (w x r)_d = eps_{d a b} w_a r_b ; d/dw_a = eps_{d a b} r_b ; d/dr_b = eps_{d a b} w_a
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    E = eps[ax]                       # (F, 3, 3): E[f, a, b] = eps_{d a b}
    dw = np.einsum("fab,fb->fa", E, r)
    dr = np.einsum("fab,a->fb", E, w)
    return dv, dw, -dr


def apply_domain_sides(grid: Grid, alpha, us):
    """Overwrite fractions / solid velocities on domain-side faces.

    WALL: alpha = 0, u_s = 0.  INFLOW: alpha = 0, u_s = inflow speed into the
    domain.  OUTFLOW: unchanged (alpha from phi; the ghost pressure is 0).
    Returns new arrays and a mask of the overridden faces.
    """
    alpha = alpha.copy()
    us = us.copy()
    side = grid.face_side()
    fixed = np.zeros(alpha.size, bool)
    for s in range(6):
        kind = grid.bc[s]
        m = side == s
        if kind == WALL:
            alpha[m] = 0.0
            us[m] = 0.0
            fixed |= m
        elif kind == INFLOW:
            alpha[m] = 0.0
            us[m] = grid.inflow_speed * (1.0 if s % 2 == 0 else -1.0)
            fixed |= m
        elif kind in (OUTFLOW, PERIODIC):
            pass
    return alpha, us, fixed


class FaceGeometry:
    """alpha and u_s on every face for a given node SDF and face solid velocity."""

    def __init__(self, grid: Grid, phi_nodes, us_faces):
        self.grid = grid
        self.corners = face_corner_nodes(grid)
        self.phi_nodes = phi_nodes
        a, da = face_fraction(phi_nodes[self.corners])
        self.alpha, self.us, self.fixed = apply_domain_sides(grid, a, us_faces)
        self.dalpha = np.where(self.fixed[:, None], 0.0, da)

    def alpha_vjp(self, galpha):
        """d J / d phi_nodes from d J / d alpha."""
        out = np.zeros(self.phi_nodes.size)
        np.add.at(out, self.corners.ravel(), (self.dalpha * galpha[:, None]).ravel())
        return out

    def alpha_jvp(self, dphi_nodes):
        return (self.dalpha * dphi_nodes[self.corners]).sum(axis=1)


def sphere_geometry(grid: Grid, spheres):
    """Static union of spheres: (FaceGeometry)."""
    phi = phi_spheres(grid.node_positions(), spheres)
    return FaceGeometry(grid, phi, np.zeros(grid.nfaces))


def no_solid_geometry(grid: Grid):
    phi = np.full(int(np.prod(grid.node_shape)), 1.0)
    return FaceGeometry(grid, phi, np.zeros(grid.nfaces))


class EllipsoidGeometry(FaceGeometry):
    """Rigid ellipsoid at pose (c, R) with semi-axes a, moving with (v, w).

    ``vjp`` maps (dJ/dalpha, dJ/du_s) to dJ/d(c, a, R, v, w); ``jvp`` the reverse.
    """

    def __init__(self, grid: Grid, c, a, R, v, w):
        self.c, self.a, self.R, self.v, self.w = (np.asarray(t, float) for t in (c, a, R, v, w))
        xn = grid.node_positions()
        phi, self.gc, self.ga, self.gR = phi_ellipsoid(xn, self.c, self.a, self.R, with_grad=True)
        us = rigid_face_velocity(grid, self.c, self.v, self.w)
        super().__init__(grid, phi, us)
        self.dv, self.dw, self.dcu = rigid_face_velocity_partials(grid, self.c, self.v, self.w)
        live = ~self.fixed
        self.dv[~live] = 0.0
        self.dw[~live] = 0.0
        self.dcu[~live] = 0.0

    def vjp(self, galpha, gus):
        gphi = self.alpha_vjp(galpha)
        gc = gphi @ self.gc + gus @ self.dcu
        ga = gphi @ self.ga
        gR = np.einsum("n,nij->ij", gphi, self.gR)
        gv = gus @ self.dv
        gw = gus @ self.dw
        return dict(c=gc, a=ga, R=gR, v=gv, w=gw)

    def jvp(self, dc, da, dR, dv, dw):
        dphi = self.gc @ dc + self.ga @ da + np.einsum("nij,ij->n", self.gR, dR)
        dalpha = self.alpha_jvp(dphi)
        dus = self.dv @ dv + self.dw @ dw + self.dcu @ dc
        return dalpha, dus
