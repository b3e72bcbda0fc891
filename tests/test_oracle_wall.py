"""Pins of the channel oracle (oracle/wall.py): the deformable B-spline wall,
its knot chain, and the outflow-flux losses."""
import numpy as np
import pytest

from oracle.geometry import face_normal_axis
from oracle.step import Step, StepParams
from oracle.wall import (ChannelRollout, WallGeometry, bspline3, bspline_basis, channel_grid,
                         constraint_net_orientation, flux_loss, outlet_mask, outlet_window, wall_time_factors)


def test_cardinal_cubic_bspline_values():
    # textbook values of the centred cubic B-spline
    s = np.array([0.0, 0.5, -0.5, 1.0, -1.0, 1.5, 2.0, -2.0, 2.5])
    ref = np.array([2 / 3, 23 / 48, 23 / 48, 1 / 6, 1 / 6, 1 / 48, 0.0, 0.0, 0.0])
    np.testing.assert_allclose(bspline3(s), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("M,L", [(16, 1.0), (32, 2.0), (5, 0.7)])
def test_bspline_partition_of_unity_and_linear_reproduction(M, L):
    s = np.linspace(0.0, L, 1001)
    B = bspline_basis(s, M, L)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    # uniform cubic B-splines reproduce linear functions: control m at (m - 1) D
    D = L / (M - 3)
    np.testing.assert_allclose(B @ ((np.arange(M) - 1.0) * D), s, rtol=0, atol=1e-13)
    assert np.all(B >= 0.0)


def test_flat_wall_fractions_are_exact():
    # all amplitudes 1: h = 1 on the whole side, so phi = x - d is planar and
    # every fraction is a clipped linear function of the face's x extent
    n, dx = (8, 6, 10), 0.125
    g = channel_grid(n, dx)
    f = 1.0
    t = 0.4   # s(t) = (1 - cos(0.8 pi)) / 2
    amp = 0.3
    geo = WallGeometry(g, np.ones((16, 32)), t, f, amp)
    s, sd = wall_time_factors(t, f)
    d = amp * s
    x = g.all_face_positions()
    ax = face_normal_axis(g)
    live = ~geo.fixed
    lo = x[:, 0] - np.where(ax == 0, 0.0, 0.5 * dx)
    want = np.where(ax == 0, (x[:, 0] > d).astype(float), np.clip((lo + dx - d) / dx, 0.0, 1.0))
    np.testing.assert_allclose(geo.alpha[live], want[live], rtol=0, atol=1e-14)
    np.testing.assert_allclose(geo.us[live & (ax == 0)], amp * sd, rtol=0, atol=1e-15)
    assert np.all(geo.us[live & (ax != 0)] == 0.0)   # (the inlet side carries the inflow speed)


def _wall(seed=0, n=(6, 6, 12), dx=1.0 / 6, t=0.35, f=1.3, amp=0.35):
    rng = np.random.default_rng(seed)
    g = channel_grid(n, dx)
    a = rng.uniform(0.0, 1.0, (16, 32))
    return g, a, t, f, amp, rng


def test_knot_chain_finite_differences_and_adjoint_identity():
    g, a, t, f, amp, rng = _wall()
    ga_w = rng.standard_normal(g.nfaces)
    gu_w = rng.standard_normal(g.nfaces)

    def J(aa):
        geo = WallGeometry(g, aa, t, f, amp)
        return float(ga_w @ geo.alpha + gu_w @ geo.us)

    geo = WallGeometry(g, a, t, f, amp)
    grad = geo.vjp(ga_w, gu_w)
    for _ in range(3):
        da = rng.standard_normal(a.shape)
        h = 1e-6
        fd = (J(a + h * da) - J(a - h * da)) / (2 * h)
        assert abs(fd - np.sum(grad * da)) <= 1e-6 * max(1.0, abs(fd))
        dal, dus = geo.jvp(da)
        assert abs(ga_w @ dal + gu_w @ dus - np.sum(grad * da)) <= 1e-12 * max(1.0, abs(fd))


def test_total_outflow_flux_is_geometry_only():
    # summing the projection's constraint over the active cells leaves the
    # outlet flux equal to the inflow plus the solid flux through faces
    # between active and inactive cells (fraction 0, so the stored velocity is
    # u_s there): the loss does not depend on the incoming velocity, and its
    # gradient w.r.t. the knots is the solid flux's derivative
    g, a, t, f, amp, rng = _wall(seed=3)
    dt = 0.5 * g.dx
    prm = StepParams(g, dt, tol=1e-13)
    geo = WallGeometry(g, a, t, f, amp)
    u0 = rng.standard_normal(g.nfaces)
    st = Step(prm, u0, geo.alpha, geo.us)
    J, lu = flux_loss(g, dt, st.result)
    D = constraint_net_orientation(g, geo.alpha)
    other = ~outlet_mask(g)
    assert np.all(geo.alpha[other & (D != 0)] == 0.0)
    c = dt * g.dx * g.dx
    closed = c * float(np.sum((D * geo.us)[other]))
    assert abs(J - closed) <= 1e-10 * abs(closed)
    assert np.any((D != 0) & other & (face_normal_axis(g) == 0) & (geo.us != 0.0))   # the wall's flux enters
    gu, g_alpha, g_us = st.vjp(lu)
    assert np.linalg.norm(gu) <= 1e-9 * np.linalg.norm(lu)
    ga = geo.vjp(g_alpha, g_us)
    gus_closed = np.where(other, c * D, 0.0)
    ga_closed = geo.vjp(np.zeros(g.nfaces), gus_closed)
    assert np.linalg.norm(ga_closed) > 0.0
    np.testing.assert_allclose(ga, ga_closed, rtol=0, atol=1e-9 * np.abs(ga_closed).max())


def test_windowed_channel_rollout_finite_differences():
    g, a, t, f, amp, rng = _wall(seed=5, amp=0.3)
    dt = 0.5 * g.dx
    prm = StepParams(g, dt, tol=1e-13)
    w = outlet_window(g, rng)
    assert np.all(w[~outlet_mask(g)] == 0.0) and w.max() > 0.0
    u0 = 0.3 * rng.standard_normal(g.nfaces)
    R = ChannelRollout(prm, u0, a, f=2.5, steps=3, amp=amp, window=w)
    R.forward()
    gu, gk = R.backward()

    def J(uu, aa):
        return ChannelRollout(prm, uu, aa, f=2.5, steps=3, amp=amp, window=w).forward(keep=False)

    h = 1e-6
    for _ in range(2):
        da = rng.standard_normal(a.shape)
        fd = (J(u0, a + h * da) - J(u0, a - h * da)) / (2 * h)
        assert abs(fd - np.sum(gk * da)) <= 2e-5 * max(abs(fd), 1e-3 * np.abs(gk).sum())
    dv = rng.standard_normal(g.nfaces)
    fd = (J(u0 + h * dv, a) - J(u0 - h * dv, a)) / (2 * h)
    assert abs(fd - gu @ dv) <= 2e-5 * max(abs(fd), 1e-12)
