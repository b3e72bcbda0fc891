"""Pins for the oracle's parametric solids (polar Bezier cross-sections,
extrusion between key sections, CSG)."""
import math

import numpy as np

from oracle import bezier as B


def _shape(rho=None, c=None, z0=-0.2, z1=0.3, o=(0.5, 0.5, 0.5), R=np.eye(3)):
    if rho is None:
        rho = np.full((B.N_KEY, 2 * B.N_SEG), 0.2)
    if c is None:
        c = np.zeros((B.N_KEY, 2))
    return np.concatenate([o, np.asarray(R).ravel(), [z0, z1], np.asarray(c).ravel(), np.asarray(rho).ravel()])


def _theta(*shapes, ops=None):
    m = len(shapes)
    ops = ops if ops is not None else [0] * m
    return np.concatenate([[m], ops, *shapes])


def _de_casteljau(P, t):
    P = [np.asarray(p, float) for p in P]
    while len(P) > 1:
        P = [(1 - t) * P[i] + t * P[i + 1] for i in range(len(P) - 1)]
    return P[0]


def test_polyline_vertices_lie_on_the_bezier_curve():
    # control points written out from the description, evaluated by de Casteljau
    rng = np.random.default_rng(0)
    c = rng.uniform(-0.05, 0.05, 2)
    rho = rng.uniform(0.1, 0.3, 2 * B.N_SEG)
    N = B.N_SEG
    ctrl = []
    for m in range(N):
        a1 = 2 * math.pi * m / N + 2 * math.pi / (3 * N)
        a2 = 2 * math.pi * (m + 1) / N - 2 * math.pi / (3 * N)
        ctrl.append((c + rho[2 * m] * np.array([math.cos(a1), math.sin(a1)]),
                     c + rho[2 * m + 1] * np.array([math.cos(a2), math.sin(a2)])))
    V = B.polyline(c[None], rho[None])[0]
    for m in range(N):
        e0 = 0.5 * (ctrl[m - 1][1] + ctrl[m][0])
        e1 = 0.5 * (ctrl[m][1] + ctrl[(m + 1) % N][0])
        for k in range(B.N_SMP):
            want = _de_casteljau([e0, ctrl[m][0], ctrl[m][1], e1], k / B.N_SMP)
            np.testing.assert_allclose(V[m * B.N_SMP + k], want, atol=1e-15)


def test_equal_radii_joints_and_symmetry():
    r = 0.2
    sh = B.unpack(_theta(_shape()))[0][0]
    # joints at polar angle 2 pi m / N and radius r cos(2 pi / (3 N)): on the surface
    N = B.N_SEG
    rj = r * math.cos(2 * math.pi / (3 * N))
    pts = np.array([[0.5 + rj * math.cos(2 * math.pi * m / N), 0.5 + rj * math.sin(2 * math.pi * m / N), 0.55]
                    for m in range(N)])
    np.testing.assert_allclose(B.shape_distance(pts, sh), 0.0, atol=1e-15)
    # N-fold symmetry about the axis, inside at the centre, outside far away
    rng = np.random.default_rng(1)
    q = rng.uniform(0.2, 0.8, (200, 3))
    q[:, 2] = rng.uniform(0.35, 0.75, 200)
    rot = q.copy()
    rot[:, 0] = 0.5 - (q[:, 1] - 0.5)
    rot[:, 1] = 0.5 + (q[:, 0] - 0.5)
    np.testing.assert_allclose(B.shape_distance(rot, sh), B.shape_distance(q, sh), atol=1e-14)
    assert B.shape_distance(np.array([[0.5, 0.5, 0.5]]), sh)[0] < 0
    assert B.shape_distance(np.array([[0.95, 0.5, 0.5]]), sh)[0] > 0


def test_caps_are_planes():
    sh = B.unpack(_theta(_shape()))[0][0]
    # above z1 over the section's interior the distance is the height over the cap
    pts = np.array([[0.5, 0.5, 0.5 + 0.3 + h] for h in (0.01, 0.05, 0.1)])
    np.testing.assert_allclose(B.shape_distance(pts, sh), [0.01, 0.05, 0.1], atol=1e-15)
    pts = np.array([[0.52, 0.49, 0.5 - 0.2 - h] for h in (0.02, 0.07)])
    np.testing.assert_allclose(B.shape_distance(pts, sh), [0.02, 0.07], atol=1e-15)


def test_csg_union_and_intersection():
    rng = np.random.default_rng(2)
    a = _shape(rho=rng.uniform(0.15, 0.25, (B.N_KEY, 2 * B.N_SEG)))
    b = _shape(rho=rng.uniform(0.1, 0.2, (B.N_KEY, 2 * B.N_SEG)), o=(0.6, 0.45, 0.5))
    x = rng.uniform(0, 1, (500, 3))
    pa, pb = B.phi_bezier(x, _theta(a)), B.phi_bezier(x, _theta(b))
    np.testing.assert_array_equal(B.phi_bezier(x, _theta(a, a)), pa)
    np.testing.assert_array_equal(B.phi_bezier(x, _theta(a, a, ops=[0, 1])), pa)
    np.testing.assert_array_equal(B.phi_bezier(x, _theta(a, b)), np.minimum(pa, pb))
    np.testing.assert_array_equal(B.phi_bezier(x, _theta(a, b, ops=[0, 1])), np.maximum(pa, pb))


def test_parameter_gradient_against_central_differences():
    rng = np.random.default_rng(3)
    ang = 0.4
    R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1.0]])
    a = _shape(rho=rng.uniform(0.15, 0.25, (B.N_KEY, 2 * B.N_SEG)), c=rng.uniform(-0.03, 0.03, (B.N_KEY, 2)),
               R=R, z0=-0.25, z1=0.2)
    b = _shape(rho=rng.uniform(0.1, 0.2, (B.N_KEY, 2 * B.N_SEG)), o=(0.62, 0.45, 0.5))
    theta = _theta(a, b)
    x = rng.uniform(0.2, 0.8, (400, 3))
    phi, G = B.phi_bezier(x, theta, with_grad=True)
    h = 1e-7
    ok = 0
    total = 0
    for p in range(3, len(theta)):
        e = np.zeros(len(theta))
        e[p] = h
        fp, fm = B.phi_bezier(x, theta + e), B.phi_bezier(x, theta - e)
        fd = (fp - fm) / (2 * h)
        # one-sided differences that disagree mark a kink (closest edge, cap or
        # CSG switch) inside the step: central differences mean nothing there
        smooth = np.abs((fp - phi) / h - (phi - fm) / h) <= 1e-5
        good = np.abs(fd - G[:, p]) <= 1e-6 + 1e-5 * np.abs(fd)
        ok += np.count_nonzero(good & smooth)
        total += np.count_nonzero(smooth)
    assert total > 0.9 * 400 * (len(theta) - 3)
    assert ok == total


def test_step_gradient_through_the_solids_against_central_differences():
    """J = <w, U^{n+1}> of one step around a two-solid scene: the adjoint chain
    (projection, fractions, the solids' parameter gradient) against central
    differences in a few parameters."""
    from oracle.mac import Grid
    from oracle.step import Step, StepParams
    import scenes
    n = 12
    g = Grid((n, n, n), 1.0 / n)
    rng = np.random.default_rng(4)
    a = _shape(rho=rng.uniform(0.15, 0.25, (B.N_KEY, 2 * B.N_SEG)), c=rng.uniform(-0.03, 0.03, (B.N_KEY, 2)))
    # no cap on a node plane (k / 12): a face lying in phi = 0 switches its fraction by a jump
    b = _shape(rho=rng.uniform(0.1, 0.18, (B.N_KEY, 2 * B.N_SEG)), o=(0.6, 0.42, 0.47))
    theta = _theta(a, b)
    u0 = scenes.curl_noise((n, n, n), 1.0 / n, rng)
    w = rng.standard_normal(g.nfaces)
    prm = StepParams(g, 0.5 / n, tol=1e-13)

    def J(th):
        geo = B.BezierGeometry(g, th)
        return w @ Step(prm, u0, geo.alpha, geo.us).result
    geo = B.BezierGeometry(g, theta)
    st = Step(prm, u0, geo.alpha, geo.us)
    _, galpha, _ = st.vjp(w)
    grad = geo.vjp(galpha)
    m = 2
    for p in [1 + m + 0, 1 + m + 12, 1 + m + 14, 1 + m + 22, 1 + m + B.SHAPE_PARAMS + 2]:
        h = 1e-6
        e = np.zeros_like(theta)
        e[p] = h
        fd = (J(theta + e) - J(theta - e)) / (2 * h)
        assert abs(fd - grad[p]) <= 2e-3 * max(abs(fd), 1e-3), (p, fd, grad[p])
