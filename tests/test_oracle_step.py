"""Pins for the oracle's full step and its adjoint."""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle.mac import Grid, PERIODIC, WALL
from oracle.advection import laplacian_faces, laplacian_periodic
from oracle.geometry import no_solid_geometry, EllipsoidGeometry
from oracle.rollout import EllipsoidRollout, octant_loss, rodrigues
from oracle.step import Step, StepParams
from tests.torch_bruteforce import TinyBox, ellipsoid_rollout_loss


def _taylor_green(n, nu, t_end, closed=False):
    # periodic box [0, 2 pi]^3, or the closed box [0, pi]^3 whose walls the
    # 2D Taylor-Green vortex crosses nowhere (u = 0 on the x walls, v = 0 on
    # the y walls; the tangential components have zero normal derivative)
    L = math.pi if closed else 2 * math.pi
    g = Grid((n, n, n), L / n, bc=(WALL,) * 6 if closed else (PERIODIC,) * 6)
    geo = no_solid_geometry(g)
    if closed:
        from oracle.geometry import apply_domain_sides
        geo.alpha, geo.us, geo.fixed = apply_domain_sides(g, np.ones(g.nfaces), np.zeros(g.nfaces))
    x = [g.face_positions(d) for d in range(3)]
    u0 = np.concatenate([np.sin(x[0][:, 0]) * np.cos(x[0][:, 1]),
                         -np.cos(x[1][:, 0]) * np.sin(x[1][:, 1]),
                         np.zeros(g.nf(2))])
    dt = 0.5 * g.dx
    steps = int(round(t_end / dt))
    prm = StepParams(g, dt, nu=nu, tol=1e-12)
    u = u0
    for _ in range(steps):
        u = Step(prm, u, geo.alpha, geo.us).result
    t = steps * dt
    exact = u0 * math.exp(-2 * nu * t)
    amp = (u @ u0) / (u0 @ u0)
    return np.linalg.norm(u - exact) / np.linalg.norm(exact), amp, math.exp(-2 * nu * t)


def test_taylor_green_decay_converges():
    nu = 0.05
    errs, amps = [], []
    for n in (8, 16, 32):
        e, amp, ref = _taylor_green(n, nu, 0.8)
        errs.append(e)
        amps.append(abs(amp - ref))
    # first-order convergence of the field and of the decay rate
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1], errs
    assert amps[2] < amps[1] < amps[0], amps
    assert errs[2] < 0.08


def test_taylor_green_decay_converges_closed_box():
    """The same first-order convergence in the closed box [0, pi]^3 with the
    face-lattice viscosity (no edge leaves the lattice at a wall)."""
    nu = 0.05
    errs, amps = [], []
    for n in (8, 16, 32):
        e, amp, ref = _taylor_green(n, nu, 0.4, closed=True)
        errs.append(e)
        amps.append(abs(amp - ref))
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1], errs
    assert amps[2] < amps[1] < amps[0], amps
    assert errs[2] < 0.08


def test_face_laplacian_periodic_equals_seven_point():
    g = Grid((6, 5, 4), 0.3, bc=(PERIODIC,) * 6)
    u = np.random.default_rng(0).standard_normal(g.nfaces)
    np.testing.assert_allclose(laplacian_faces(g, u), laplacian_periodic(g, u), rtol=0, atol=1e-12)


def test_face_laplacian_closed_box_modes_and_symmetry():
    """In the closed box the Taylor-Green modes are eigenvectors of the face
    Laplacian at every lattice point off the normal component's boundary
    faces, with the 1D eigenvalue -(2 - 2 cos h) / h^2 per varying axis
    (closed form); the operator is symmetric and annihilates constants."""
    n = 12
    h = math.pi / n
    g = Grid((n, n, n), h)
    x = [g.face_positions(d) for d in range(3)]
    u = np.concatenate([np.sin(x[0][:, 0]) * np.cos(x[0][:, 1]) * np.cos(2 * x[0][:, 2]),
                        -np.cos(x[1][:, 0]) * np.sin(x[1][:, 1]) * np.cos(2 * x[1][:, 2]),
                        np.zeros(g.nf(2))])
    lam = -(2 * (2 - 2 * math.cos(h)) + (2 - 2 * math.cos(2 * h))) / h ** 2
    Lu = laplacian_faces(g, u)
    inner = np.ones(g.nfaces, bool)
    for d in range(2):      # the u and v boundary faces along their own axis
        off = g.face_offset(d)
        own = np.rint(x[d][:, d] / h).astype(int)
        inner[off:off + g.nf(d)] &= (own > 0) & (own < n)
    np.testing.assert_allclose(Lu[inner], lam * u[inner], rtol=0, atol=1e-9 * abs(lam))
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(g.nfaces), rng.standard_normal(g.nfaces)
    assert abs(laplacian_faces(g, a) @ b - a @ laplacian_faces(g, b)) <= 1e-10 * abs(a @ laplacian_faces(g, b))
    assert np.abs(laplacian_faces(g, np.full(g.nfaces, 3.0))).max() == 0.0


def test_step_adjoint_identity_with_moving_solid():
    n = 10
    g = Grid((n, n, n), 1.0 / n)
    rng = np.random.default_rng(7)
    u = scenes.curl_noise(g.n, g.dx, rng)
    prm = StepParams(g, 0.5 * g.dx, tol=1e-13)
    c, a = np.array([0.52, 0.47, 0.5]), np.array([0.25, 0.18, 0.3])
    R = rodrigues(np.array([0.3, 0.9, -0.4]))
    v, w = rng.uniform(-0.5, 0.5, 3), rng.uniform(-0.5, 0.5, 3)
    geo = EllipsoidGeometry(g, c, a, R, v, w)
    st = Step(prm, u, geo.alpha, geo.us)
    du = rng.standard_normal(g.nfaces)
    tang = [rng.standard_normal(3), rng.standard_normal(3), rng.standard_normal((3, 3)),
            rng.standard_normal(3), rng.standard_normal(3)]
    dalpha, dus = geo.jvp(*tang)
    jv = st.jvp(du, dalpha, dus)
    wv = rng.standard_normal(g.nfaces)
    gu, galpha, gus = st.vjp(wv)
    d = geo.vjp(galpha, gus)
    lhs = jv @ wv
    rhs = (gu @ du + d["c"] @ tang[0] + d["a"] @ tang[1] + np.sum(d["R"] * tang[2])
           + d["v"] @ tang[3] + d["w"] @ tang[4])
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


def test_hand_adjoint_matches_autograd_bruteforce():
    n = 6
    sc = scenes.scene_ellipsoid_rollout(seed=2, n=n, steps=2)
    sc.theta0[3:6] = [0.3, 0.22, 0.26]           # large enough to cut faces at this size
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, method="dense")
    ro = EllipsoidRollout(prm, sc.u0, sc.theta0, sc.ctrl)
    J, gT = octant_loss(g, ro.forward())
    gu, gth, gctrl = ro.backward(gT)

    box = TinyBox(sc.n, sc.dx)
    u0 = torch.tensor(sc.u0, requires_grad=True)
    th = torch.tensor(sc.theta0, requires_grad=True)
    ct = torch.tensor(sc.ctrl, requires_grad=True)
    Jt = ellipsoid_rollout_loss(box, u0, th, ct, sc.dt)
    Jt.backward()
    assert abs(Jt.item() - J) <= 1e-12 * abs(J)
    np.testing.assert_allclose(gu, u0.grad.numpy(), rtol=1e-9, atol=1e-11 * np.abs(gu).max())
    np.testing.assert_allclose(gth, th.grad.numpy(), rtol=1e-8, atol=1e-10 * np.abs(gth).max())
    np.testing.assert_allclose(gctrl, ct.grad.numpy(), rtol=1e-8, atol=1e-10 * np.abs(gctrl).max())
