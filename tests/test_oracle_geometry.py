"""Pins for the oracle's geometry: face fractions, signed distances, solid velocity."""
import json
import os

import numpy as np
import pytest

from oracle.mac import Grid, gradient_matrix
from oracle.geometry import (face_fraction, phi_ellipsoid, phi_spheres, rigid_face_velocity,
                             EllipsoidGeometry, face_corner_nodes)
from oracle.rollout import rodrigues

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_printed_triangle_case():
    cases = json.load(open(os.path.join(GOLD, "alpha_triangle.json")))["cases"]
    phis = np.array([c["phi"] for c in cases])
    alpha, _ = face_fraction(phis)
    np.testing.assert_allclose(alpha, [c["alpha"] for c in cases], rtol=0, atol=1e-15)


def _clip_area(phi_fn):
    """Exact fluid area of the unit square {phi > 0} for an affine phi, by
    Sutherland-Hodgman clipping of the square against the half-plane (an
    independent brute force of the marching-squares areas)."""
    poly = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    out = []
    for a, b in zip(poly, poly[1:] + poly[:1]):
        fa, fb = phi_fn(*a), phi_fn(*b)
        if fa > 0:
            out.append(a)
        if (fa > 0) != (fb > 0):
            t = fa / (fa - fb)
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    if len(out) < 3:
        return 0.0
    x = np.array([p[0] for p in out])
    y = np.array([p[1] for p in out])
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def test_planar_phi_gives_exact_area():
    rng = np.random.default_rng(0)
    corners = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]    # cyclic A, B, C, D
    phis, exact = [], []
    for _ in range(2000):
        g = rng.standard_normal(2)
        c0 = rng.uniform(-1.5, 1.5)
        fn = lambda x, y: g[0] * x + g[1] * y + c0
        phis.append([fn(*p) for p in corners])
        exact.append(_clip_area(fn))
    alpha, _ = face_fraction(np.array(phis))
    np.testing.assert_allclose(alpha, exact, rtol=0, atol=1e-13)
    # all corner-count cases are covered
    cnt = (np.array(phis) > 0).sum(axis=1)
    assert set(cnt.tolist()) == {0, 1, 2, 3, 4}


def test_complement_and_extremes():
    rng = np.random.default_rng(1)
    phis = rng.standard_normal((5000, 4))
    fluid = phis > 0
    diag = (fluid[:, 0] == fluid[:, 2]) & (fluid[:, 1] == fluid[:, 3]) & (fluid[:, 0] != fluid[:, 1])
    a1, _ = face_fraction(phis)
    a2, _ = face_fraction(-phis)
    np.testing.assert_allclose((a1 + a2)[~diag], 1.0, atol=1e-14)
    assert np.all((a1 >= 0) & (a1 <= 1))
    np.testing.assert_array_equal(face_fraction(np.abs(phis) + 0.1)[0], 1.0)
    np.testing.assert_array_equal(face_fraction(-np.abs(phis))[0], 0.0)


def test_saddle_reading():
    # connected when the corner mean is positive: 1 - two solid triangles
    a, _ = face_fraction(np.array([[2.0, -1.0, 2.0, -1.0]]))
    t = 1.0 / 3.0                               # solid share along each edge from B or D
    assert abs(a[0] - (1.0 - 2 * 0.5 * t * t)) < 1e-15
    a, _ = face_fraction(np.array([[1.0, -2.0, 1.0, -2.0]]))
    assert abs(a[0] - 2 * 0.5 * t * t) < 1e-15


def test_fraction_gradient_fd():
    rng = np.random.default_rng(2)
    phis = rng.standard_normal((3000, 4))
    _, g = face_fraction(phis)
    h = 1e-7
    for k in range(4):
        e = np.zeros(4)
        e[k] = h
        ap, _ = face_fraction(phis + e)
        am, _ = face_fraction(phis - e)
        fd = (ap - am) / (2 * h)
        same = ((phis + e > 0) == (phis - e > 0)).all(axis=1)
        # skip configurations where the saddle decision flips inside the FD stencil
        same &= np.sign((phis + e).mean(axis=1)) == np.sign((phis - e).mean(axis=1))
        np.testing.assert_allclose(g[same, k], fd[same], atol=2e-6, rtol=1e-5)


def test_ellipsoid_reduces_to_sphere_and_gradients():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (500, 3))
    c = np.array([0.4, 0.55, 0.5])
    R = rodrigues(np.array([0.3, -1.1, 0.7]))
    r = 0.17
    phi = phi_ellipsoid(x, c, np.full(3, r), R)
    np.testing.assert_allclose(phi, np.linalg.norm(x - c, axis=1) - r, atol=1e-14)
    np.testing.assert_allclose(phi_spheres(x, np.array([[*c, r]])), phi, atol=1e-14)
    # zero set is the ellipsoid surface for unequal axes
    a = np.array([0.1, 0.15, 0.2])
    dirs = rng.standard_normal((200, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    surf = c + (dirs * a) @ R.T
    np.testing.assert_allclose(phi_ellipsoid(surf, c, a, R), 0.0, atol=1e-14)
    # partials against central differences
    _, gc, ga, gR = phi_ellipsoid(x, c, a, R, with_grad=True)
    h = 1e-7
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd = (phi_ellipsoid(x, c + e, a, R) - phi_ellipsoid(x, c - e, a, R)) / (2 * h)
        np.testing.assert_allclose(gc[:, i], fd, atol=1e-6)
        fd = (phi_ellipsoid(x, c, a + e, R) - phi_ellipsoid(x, c, a - e, R)) / (2 * h)
        np.testing.assert_allclose(ga[:, i], fd, atol=1e-5, rtol=1e-6)
        for j in range(3):
            E = np.zeros((3, 3))
            E[i, j] = h
            fd = (phi_ellipsoid(x, c, a, R + E) - phi_ellipsoid(x, c, a, R - E)) / (2 * h)
            np.testing.assert_allclose(gR[:, i, j], fd, atol=1e-6)


def test_rigid_velocity_is_discretely_divergence_free():
    g = Grid((9, 7, 8), 1.0 / 8)
    G = gradient_matrix(g)
    us = rigid_face_velocity(g, np.array([0.3, 0.2, 0.6]), np.array([0.4, -0.2, 0.9]),
                             np.array([1.3, -0.7, 0.25]))
    # midpoint sampling is exact for linear fields; a rigid field has zero divergence
    np.testing.assert_allclose(G.T @ us, 0.0, atol=1e-13)


def test_geometry_vjp_jvp_adjoint_identity():
    g = Grid((10, 10, 10), 0.1)
    rng = np.random.default_rng(4)
    c = np.array([0.48, 0.52, 0.5])
    a = np.array([0.22, 0.3, 0.18])
    R = rodrigues(np.array([0.4, 0.2, -0.9]))
    v = rng.uniform(-0.5, 0.5, 3)
    w = rng.uniform(-0.5, 0.5, 3)
    geo = EllipsoidGeometry(g, c, a, R, v, w)
    assert 0 < np.count_nonzero((geo.alpha > 0) & (geo.alpha < 1))
    ga, gu = rng.standard_normal(g.nfaces), rng.standard_normal(g.nfaces)
    d = geo.vjp(ga, gu)
    t = [rng.standard_normal(3), rng.standard_normal(3), rng.standard_normal((3, 3)),
         rng.standard_normal(3), rng.standard_normal(3)]
    da, du = geo.jvp(*t)
    lhs = da @ ga + du @ gu
    rhs = d["c"] @ t[0] + d["a"] @ t[1] + np.sum(d["R"] * t[2]) + d["v"] @ t[3] + d["w"] @ t[4]
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # and the tangent against finite differences of alpha and u_s
    h = 1e-7
    gp = EllipsoidGeometry(g, c + h * t[0], a + h * t[1], R + h * t[2], v + h * t[3], w + h * t[4])
    gm = EllipsoidGeometry(g, c - h * t[0], a - h * t[1], R - h * t[2], v - h * t[3], w - h * t[4])
    np.testing.assert_allclose(da, (gp.alpha - gm.alpha) / (2 * h), atol=1e-5)
    np.testing.assert_allclose(du, (gp.us - gm.us) / (2 * h), atol=1e-7)


def test_corner_nodes_are_the_face_corners():
    g = Grid((3, 4, 5), 0.25)
    xn = g.node_positions()
    cn = face_corner_nodes(g)
    xf = g.all_face_positions()
    centre = xn[cn].mean(axis=1)
    np.testing.assert_allclose(centre, xf, atol=1e-15)
    # consecutive corners share an edge of length dx (cyclic order)
    for k in range(4):
        d = np.linalg.norm(xn[cn[:, k]] - xn[cn[:, (k + 1) % 4]], axis=1)
        np.testing.assert_allclose(d, 0.25, atol=1e-15)


def test_moving_ellipsoid_cut_cells_exceed_fp16_range():
    # why the finest multigrid level keeps 1/diag in FP32 when the rest of the
    # V-cycle is stored in 2 bytes: at 128^3 the moving-ellipsoid scene has cut
    # cells nearly inside the body whose diagonal (the sum of their face
    # fractions) is below 1/65504, and fractions below FP16's smallest normal
    import scenes
    from oracle.mac import Grid
    from oracle.rollout import EllipsoidRollout
    from oracle.step import StepParams
    n = 128
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=n, steps=33)
    g = Grid(sc.n, sc.dx)
    c, R = EllipsoidRollout(StepParams(g, sc.dt), sc.u0, sc.theta0, sc.ctrl).poses()[32]
    al = EllipsoidGeometry(g, c, sc.theta0[3:6], R, sc.ctrl[32, :3], sc.ctrl[32, 3:]).alpha
    fx = al[:g.nf(0)].reshape(n, n, n + 1)
    fy = al[g.nf(0):g.nf(0) + g.nf(1)].reshape(n, n + 1, n)
    fz = al[g.nf(0) + g.nf(1):].reshape(n + 1, n, n)
    diag = fx[:, :, :-1] + fx[:, :, 1:] + fy[:, :-1, :] + fy[:, 1:, :] + fz[:-1] + fz[1:]
    tiny = (diag > 0) & (diag < 1.0 / 65504.0)
    assert 0 < tiny.sum() < 100
    assert np.sum((al > 0) & (al < 6.1e-5)) > 0
