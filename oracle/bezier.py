"""Parametric solids of the paper's geometry representation: closed polar
Bezier cross-sections, extruded between key cross-sections, combined by CSG
union / intersection (FP64 oracle; test infrastructure only).

Paper, Sec. Geometry Representation and App. "Geometry Representation
Implementation":

* a closed 2D curve is N cubic Bezier segments around a centre c; segment m
  spans the polar angles [2 pi m / N, 2 pi (m + 1) / N]; its two inner
  control points sit 2 pi / (3N) inside that span at polar distances rho_1^m
  and rho_2^m from c; consecutive segments share an end point collinear with
  the two control points around it;
* a 3D solid is a list of such cross-sections (centres and control radii)
  along the z axis of its own frame, evenly spaced between z0 and z1; the
  cross-section at any z interpolates the key ones;
* solids combine by CSG union and intersection.

Readings (the paper leaves them open; the GPU path follows the same ones):

* the shared end point is the midpoint of the two control points around it
  (the collinearity the paper asks for, with the joint halfway);
* the curve is taken as its polyline through S = 16 points per segment
  (t = k / S), so that the signed distance is exact and cheap on both sides;
* between key cross-sections (s = (z - z0) / (z1 - z0) in [0, 1], keys at
  s = i / (K - 1)) the centre and radii are interpolated linearly, clamped
  outside [0, 1] (the printed interpolation formula is a power series in s
  that does not pass through the key cross-sections; linear interpolation is
  what "interpolates the key cross-sections" asks);
* the solid's signed distance (negative inside) in its frame p = R^T (x - o)
  is max(d2(p_x, p_y), z0 - p_z, p_z - z1), d2 the signed distance to the
  cross-section's polyline (negative inside, by crossing parity); the fluid
  SDF phi (positive in fluid) of a CSG tree is the min (union) or max
  (intersection) of the solids' distances, applied left to right;
* the solids are static (u_s = 0).

Parameters of one solid (SHAPE_PARAMS = 44, in this order): frame origin o
(3), rotation R (9, row-major, body -> world), z0, z1, K = 3 key centres
(2 each), then K x 2N = 3 x 8 control radii (key-major; within a key, segment
m's two radii at 2m, 2m + 1).  A scene: theta = [m, op_1 .. op_m, shape_1 ..
shape_m], op 0 = union, 1 = intersection (op_1 is ignored).

Pinned by: tests/test_oracle_bezier.py (the curve passes exactly through its
joints, which are closed-form for equal radii; N-fold symmetry; cap faces;
CSG identities; the analytic parameter gradient against central differences).
"""
from __future__ import annotations

import math

import numpy as np

N_SEG = 4                       # Bezier segments per cross-section
N_SMP = 16                      # polyline points per segment
N_KEY = 3                       # key cross-sections
SHAPE_PARAMS = 3 + 9 + 2 + 2 * N_KEY + 2 * N_SEG * N_KEY
N_VERT = N_SEG * N_SMP


def unpack(theta):
    """theta -> (list of shape dicts, list of ops)."""
    theta = np.asarray(theta, float)
    m = int(round(theta[0]))
    ops = [int(round(v)) for v in theta[1:1 + m]]
    shapes = []
    for q in range(m):
        s = theta[1 + m + q * SHAPE_PARAMS: 1 + m + (q + 1) * SHAPE_PARAMS]
        shapes.append(dict(o=s[0:3], R=s[3:12].reshape(3, 3), z0=s[12], z1=s[13],
                           c=s[14:14 + 2 * N_KEY].reshape(N_KEY, 2),
                           rho=s[14 + 2 * N_KEY:].reshape(N_KEY, 2 * N_SEG)))
    return shapes, ops


def control_angles():
    """Polar angles of the two inner control points of every segment."""
    base = 2.0 * math.pi * np.arange(N_SEG) / N_SEG
    off = 2.0 * math.pi / (3.0 * N_SEG)
    return np.stack([base + off, base + 2.0 * math.pi / N_SEG - off], axis=1).ravel()   # (2N,)


def vertex_weights():
    """W (N_VERT, 2N): polyline vertex k = c + sum_r W[k, r] rho_r dir_r (dir_r the
    unit vector at control angle r).  Bernstein weights of the 4 points of a
    segment, with each joint the mean of the two control points around it."""
    W = np.zeros((N_VERT, 2 * N_SEG))
    for m in range(N_SEG):
        p1, p2 = 2 * m, 2 * m + 1
        prev_p2 = (2 * m - 1) % (2 * N_SEG)        # joint at the segment's start: (P2_{m-1} + P1_m) / 2
        next_p1 = (2 * m + 2) % (2 * N_SEG)        # joint at its end: (P2_m + P1_{m+1}) / 2
        for k in range(N_SMP):
            t = k / N_SMP
            b0, b1, b2, b3 = (1 - t) ** 3, 3 * (1 - t) ** 2 * t, 3 * (1 - t) * t ** 2, t ** 3
            row = W[m * N_SMP + k]
            row[prev_p2] += 0.5 * b0
            row[p1] += 0.5 * b0 + b1
            row[p2] += b2 + 0.5 * b3
            row[next_p1] += 0.5 * b3
    return W


_W = vertex_weights()
_ANG = control_angles()
_DIR = np.stack([np.cos(_ANG), np.sin(_ANG)], axis=1)                  # (2N, 2)


def section(shape, s):
    """Centre (n, 2), radii (n, 2N) at s (n,), and the key interpolation:
    key index i (n,), weight lam (n,) of key i + 1, and whether s was clamped."""
    u = np.clip(s, 0.0, 1.0) * (N_KEY - 1)
    i = np.minimum(np.floor(u).astype(int), N_KEY - 2)
    lam = u - i
    c = (1 - lam)[:, None] * shape["c"][i] + lam[:, None] * shape["c"][i + 1]
    rho = (1 - lam)[:, None] * shape["rho"][i] + lam[:, None] * shape["rho"][i + 1]
    clamped = (s < 0.0) | (s > 1.0)
    return c, rho, i, lam, clamped


def polyline(c, rho):
    """Vertices (n, N_VERT, 2) of the cross-sections with centres c (n, 2), radii rho (n, 2N)."""
    return c[:, None, :] + np.einsum("kr,nr,rd->nkd", _W, rho, _DIR)


def signed_distance_2d(q, V):
    """Signed distance of points q (n, 2) to closed polylines V (n, M, 2)
    (negative inside, by crossing parity), with the closest edge and the
    parameter tau in [0, 1] along it."""
    a = V
    b = np.roll(V, -1, axis=1)
    ab = b - a
    aq = q[:, None, :] - a
    den = np.einsum("nmd,nmd->nm", ab, ab)
    tau = np.clip(np.einsum("nmd,nmd->nm", aq, ab) / den, 0.0, 1.0)
    diff = aq - tau[..., None] * ab
    d2 = np.einsum("nmd,nmd->nm", diff, diff)
    e = np.argmin(d2, axis=1)
    n = np.arange(q.shape[0])
    dist = np.sqrt(d2[n, e])
    # crossing parity of the ray from q along +x
    ay, by = a[..., 1], b[..., 1]
    cross = (ay > q[:, None, 1]) != (by > q[:, None, 1])
    xint = a[..., 0] + (q[:, None, 1] - ay) * ab[..., 0] / np.where(by != ay, by - ay, 1.0)
    inside = (np.count_nonzero(cross & (q[:, None, 0] < xint), axis=1) % 2) == 1
    return np.where(inside, -dist, dist), e, tau[n, e], inside


def shape_distance(x, shape, with_grad=False):
    """Signed distance of the solid (negative inside) at points x (n, 3), and
    with_grad: its derivative w.r.t. the shape's 44 parameters (n, 44)."""
    o, R, z0, z1 = shape["o"], shape["R"], shape["z0"], shape["z1"]
    r = x - o[None, :]
    p = r @ R                                  # p_j = sum_i r_i R_ij (= R^T r)
    L = z1 - z0
    s = (p[:, 2] - z0) / L
    c, rho, i, lam, clamped = section(shape, s)
    V = polyline(c, rho)
    d2, e, tau, inside = signed_distance_2d(p[:, :2], V)
    cap_lo, cap_hi = z0 - p[:, 2], p[:, 2] - z1
    val = np.maximum(d2, np.maximum(cap_lo, cap_hi))
    if not with_grad:
        return val
    n = x.shape[0]
    G = np.zeros((n, SHAPE_PARAMS))
    use_d2 = d2 >= np.maximum(cap_lo, cap_hi)
    use_lo = ~use_d2 & (cap_lo >= cap_hi)
    use_hi = ~use_d2 & ~use_lo
    # d2 = sgn |q - Q|, Q = (1 - tau) a + tau b: d d2 / d Q = -sgn (q - Q) / |q - Q|
    idx = np.arange(n)
    a = V[idx, e]
    b = V[idx, (e + 1) % N_VERT]
    Q = a + tau[:, None] * (b - a)
    dq = p[:, :2] - Q
    dist = np.linalg.norm(dq, axis=1)
    sgn = np.where(inside, -1.0, 1.0)
    nvec = np.where(dist[:, None] > 0, dq / np.where(dist > 0, dist, 1.0)[:, None], 0.0) * sgn[:, None]
    # derivative w.r.t. the section's centre (every vertex moves with it) and radii
    g_c = -nvec                                                    # (n, 2)
    wa = _W[e]                                                     # (n, 2N)
    wb = _W[(e + 1) % N_VERT]
    wq = (1 - tau)[:, None] * wa + tau[:, None] * wb               # dQ/drho_r = wq_r dir_r
    g_rho = -wq * (nvec @ _DIR.T)                                  # (n, 2N)
    # through the key interpolation
    for key, wk in ((i, 1 - lam), (i + 1, lam)):
        for a_ in range(2):
            np.add.at(G, (idx, 14 + 2 * key + a_), np.where(use_d2, wk * g_c[:, a_], 0.0))
        for r_ in range(2 * N_SEG):
            np.add.at(G, (idx, 14 + 2 * N_KEY + 2 * N_SEG * key + r_), np.where(use_d2, wk * g_rho[:, r_], 0.0))
    # d d2 / d s through the interpolated section (0 where s is clamped)
    dc_ds = (shape["c"][i + 1] - shape["c"][i]) * (N_KEY - 1)
    drho_ds = (shape["rho"][i + 1] - shape["rho"][i]) * (N_KEY - 1)
    dd2_ds = np.where(clamped, 0.0, np.einsum("nd,nd->n", g_c, dc_ds) + np.einsum("nr,nr->n", g_rho, drho_ds))
    # value w.r.t. p (body frame) and the caps
    gp = np.zeros((n, 3))
    gp[:, :2] = np.where(use_d2[:, None], nvec, 0.0)
    gp[:, 2] = np.where(use_d2, dd2_ds / L, np.where(use_lo, -1.0, 1.0))
    # z0, z1: the caps directly; d2 through s = (p_z - z0) / L
    G[:, 12] = np.where(use_d2, dd2_ds * (s - 1.0) / L, np.where(use_lo, 1.0, 0.0))
    G[:, 13] = np.where(use_d2, -dd2_ds * s / L, np.where(use_hi, -1.0, 0.0))
    # frame: p = R^T (x - o)
    G[:, 0:3] = -(gp @ R.T)
    G[:, 3:12] = (r[:, :, None] * gp[:, None, :]).reshape(n, 9)
    return val, G


def phi_bezier(x, theta, with_grad=False):
    """Fluid SDF (positive in fluid) of the CSG scene at points x (n, 3); with
    with_grad also d phi / d theta (n, len(theta)), zero for m and the ops."""
    shapes, ops = unpack(theta)
    m = len(shapes)
    vals, grads = [], []
    for sh in shapes:
        if with_grad:
            v, g = shape_distance(x, sh, True)
            grads.append(g)
        else:
            v = shape_distance(x, sh)
        vals.append(v)
    phi = vals[0].copy()
    active = np.zeros(x.shape[0], int)
    for q in range(1, m):
        take = (vals[q] < phi) if ops[q] == 0 else (vals[q] > phi)
        phi = np.where(take, vals[q], phi)
        active = np.where(take, q, active)
    if not with_grad:
        return phi
    G = np.zeros((x.shape[0], len(theta)))
    for q in range(m):
        sel = active == q
        G[sel, 1 + m + q * SHAPE_PARAMS: 1 + m + (q + 1) * SHAPE_PARAMS] = grads[q][sel]
    return phi, G


class BezierGeometry:
    """Face fractions of a static CSG scene of parametric solids (u_s = 0),
    and the chain from dJ/dalpha to dJ/dtheta."""

    def __init__(self, grid, theta):
        from .geometry import FaceGeometry
        self.theta = np.asarray(theta, float)
        phi, self.G = phi_bezier(grid.node_positions(), self.theta, with_grad=True)
        self.faces = FaceGeometry(grid, phi, np.zeros(grid.nfaces))
        self.alpha, self.us, self.fixed = self.faces.alpha, self.faces.us, self.faces.fixed
        self.phi_nodes = phi

    def vjp(self, galpha, gus=None):
        """dJ/dtheta (zero for the count and the CSG ops)."""
        return self.faces.alpha_vjp(galpha) @ self.G
