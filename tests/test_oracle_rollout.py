"""Pins for the oracle's rollout adjoint (BPTT through the pose dynamics)."""
import numpy as np

import scenes
from oracle.mac import Grid
from oracle.rollout import (EllipsoidRollout, StaticRollout, octant_loss, rodrigues,
                            rodrigues_grad)
from oracle.step import StepParams


def test_rodrigues_is_a_rotation_and_its_derivative():
    rng = np.random.default_rng(0)
    for _ in range(20):
        r = rng.standard_normal(3) * rng.uniform(0.001, 3.0)
        R = rodrigues(r)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        # R rotates about r by |r|: r is fixed
        np.testing.assert_allclose(R @ r, r, atol=1e-14)
        dR = rodrigues_grad(r)
        h = 1e-6
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            np.testing.assert_allclose(dR[i], (rodrigues(r + e) - rodrigues(r - e)) / (2 * h), atol=1e-9)


def _loss(prm, grid, u0, th, ctrl):
    ro = EllipsoidRollout(prm, u0, th, ctrl)
    return octant_loss(grid, ro.forward(keep=False))[0]


def test_rollout_gradient_matches_central_differences():
    n, T = 10, 3
    sc = scenes.scene_ellipsoid_rollout(seed=1, n=n, steps=T)
    sc.theta0[3:6] = [0.24, 0.2, 0.28]
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-13)
    ro = EllipsoidRollout(prm, sc.u0, sc.theta0, sc.ctrl)
    _, gT = octant_loss(g, ro.forward())
    gu, gth, gctrl = ro.backward(gT)
    h = 1e-6
    fd = []
    for i in range(9):
        e = np.zeros(9)
        e[i] = h
        fd.append((_loss(prm, g, sc.u0, sc.theta0 + e, sc.ctrl)
                   - _loss(prm, g, sc.u0, sc.theta0 - e, sc.ctrl)) / (2 * h))
    np.testing.assert_allclose(gth, fd, rtol=1e-5, atol=1e-6 * np.abs(gth).max())
    for (s, j) in [(0, 0), (0, 4), (1, 2), (2, 5), (2, 3)]:
        e = np.zeros_like(sc.ctrl)
        e[s, j] = h
        f = (_loss(prm, g, sc.u0, sc.theta0, sc.ctrl + e) - _loss(prm, g, sc.u0, sc.theta0, sc.ctrl - e)) / (2 * h)
        assert abs(f - gctrl[s, j]) <= 1e-5 * max(abs(f), 1e-3 * np.abs(gctrl).max())
    v = np.random.default_rng(5).standard_normal(g.nfaces)
    f = (_loss(prm, g, sc.u0 + h * v, sc.theta0, sc.ctrl) - _loss(prm, g, sc.u0 - h * v, sc.theta0, sc.ctrl)) / (2 * h)
    assert abs(f - gu @ v) <= 1e-6 * abs(f)


def test_static_rollout_gradient_wrt_initial_velocity():
    sc = scenes.scene_sphere_rollout(seed=3, n=12, steps=3)
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-13)
    ro = StaticRollout(prm, sc.u0, sc.spheres)
    J, gT = octant_loss(g, ro.forward(3))
    gu = ro.backward(gT)
    v = np.random.default_rng(6).standard_normal(g.nfaces)
    h = 1e-6
    jp = octant_loss(g, StaticRollout(prm, sc.u0 + h * v, sc.spheres).forward(3, keep=False))[0]
    jm = octant_loss(g, StaticRollout(prm, sc.u0 - h * v, sc.spheres).forward(3, keep=False))[0]
    assert abs((jp - jm) / (2 * h) - gu @ v) <= 1e-6 * abs(gu @ v)
