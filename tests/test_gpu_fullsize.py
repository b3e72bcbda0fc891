"""Checks at the full sizes of the benchmark and of the precision configuration,
where the FP64 oracle cannot solve the whole system in a test: the 128^3
moving-ellipsoid step as bench.py runs it (FP16 V-cycle) against the oracle's
geometry and advection, its projection against the FP64 residual of the
oracle's operator and the update formula face by face, the adjoint of
that step against central differences, and the 256^3 twenty-sphere
projection in both V-cycle precisions against the FP64 residual of the
oracle's operator.  Every bound is tolerance + what FP32 storage of the
outputs can add (derived below)."""
import numpy as np
import pytest
import torch

import scenes
from oracle.advection import Advection
from oracle.geometry import EllipsoidGeometry
from oracle.mac import Grid
from oracle.projection import Operators
from paper_2405_14903_amd.sim import Sim, ellipsoid_poses
from tests.gpu_common import announce, dev, ellipsoid_cfg, ellipsoid_step_params, host, sphere_cfg

pytestmark = pytest.mark.gpu

EPS32 = float(np.finfo(np.float32).eps)


def test_ellipsoid_step_128_fullsize():
    announce("full size: 128^3 moving-ellipsoid step, FP16 V-cycle")
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=128, steps=1)
    g = Grid(sc.n, sc.dx)
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    tol = 1e-6
    with Sim(ellipsoid_cfg(sc.n, tol=tol, precision="fp16")) as sim:
        u0 = dev(sc.u0)
        alpha = torch.empty(g.nfaces, dtype=torch.float32, device="cuda")
        sim.set_geometry(poses[0], sc.ctrl[0], alpha_out=alpha)
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u1, st = sim.step(u0, poses[0], sc.ctrl[0], p_out=P)
        torch.cuda.synchronize()
    announce(f"  solve: {st}")
    assert st["converged"] and st["true_rel_res"] <= tol
    al, u1h, Ph = host(alpha), host(u1), host(P)
    assert np.isfinite(u1h).all()

    # geometry at full size against the oracle (same bound as at 32^3)
    c, a, R, v, w = ellipsoid_step_params(poses[0], sc.ctrl[0])
    geo = EllipsoidGeometry(g, c, a, R, v, w)
    assert np.array_equal(al > 0, geo.alpha > 0)
    np.testing.assert_allclose(al, geo.alpha, atol=1e-7, rtol=0)
    announce("  fractions match the oracle")

    # advection: on faces at least half open, the update U1 = a (U^ - k G P) +
    # (1 - a) Us gives back the advected U^, compared with the oracle's; FP32
    # storage of U1 and P adds at most eps * (|U1| / a + k (|P+| + |P-|)) per face
    k = sc.dt / sc.dx
    ops = Operators(g, al.astype(np.float64))
    adv = Advection(g, sc.u0, sc.dt)
    uh_o = adv.result
    gp = ops.G @ Ph
    openf = al >= 0.5
    uh_g = (u1h - (1.0 - al) * geo.us) / np.where(openf, al, 1.0) + k * gp
    diff = np.linalg.norm((uh_g - uh_o)[openf])
    pabs = abs(ops.G) @ np.abs(Ph)
    bound = 1e-5 * np.linalg.norm(uh_o[openf]) + 2 * EPS32 * np.linalg.norm(
        (np.abs(u1h) / np.where(openf, al, 1.0) + k * pabs)[openf])
    announce(f"  advected field on open faces: |diff| {diff:.3e} (bound {bound:.3e}, |U^| {np.linalg.norm(uh_o[openf]):.3e})")
    assert diff <= bound


def test_ellipsoid_projection_128_fullsize():
    announce("full size: 128^3 projection with the moving ellipsoid, FP16 V-cycle")
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=128, steps=1)
    g = Grid(sc.n, sc.dx)
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    tol = 1e-6
    with Sim(ellipsoid_cfg(sc.n, tol=tol, precision="fp16")) as sim:
        alpha = torch.empty(g.nfaces, dtype=torch.float32, device="cuda")
        sim.set_geometry(poses[0], sc.ctrl[0], alpha_out=alpha)
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u1, st = sim.project(dev(sc.u0), poses[0], sc.ctrl[0], p_out=P)
        torch.cuda.synchronize()
    announce(f"  solve: {st}")
    assert st["converged"]
    al, u1h, Ph = host(alpha).astype(np.float64), host(u1), host(P)
    c, a, R, v, w = ellipsoid_step_params(poses[0], sc.ctrl[0])
    us = EllipsoidGeometry(g, c, a, R, v, w).us
    u0 = sc.u0.astype(np.float32).astype(np.float64)   # the input as the GPU holds it
    k = sc.dt / sc.dx
    ops = Operators(g, al)
    # FP64 residual of the returned pressure (Eq. projection_matrix, unit
    # scale): FP32 storage of P adds at most |A| eps |P|, |A| <= 12
    b = (ops.GT @ (al * u0 + (1.0 - al) * us)) / k
    act = ops.active
    rel = np.linalg.norm(np.where(act, b - ops.apply(Ph), 0.0)) / np.linalg.norm(np.where(act, b, 0.0))
    bound = 1.5 * tol + 12.0 * EPS32 * np.linalg.norm(Ph) / np.linalg.norm(np.where(act, b, 0.0))
    announce(f"  FP64 relative residual {rel:.3e} (bound {bound:.3e})")
    assert rel <= bound
    # the update on every face (Eq. u_next_matrix), evaluated by the oracle's
    # formula from the returned P; FP32 arithmetic on the face terms adds a
    # few eps of their magnitudes
    ref = al * (u0 - k * (ops.G @ Ph)) + (1.0 - al) * us
    mag = al * (np.abs(u0) + k * (abs(ops.G) @ np.abs(Ph))) + (1.0 - al) * np.abs(us)
    err = np.abs(u1h - ref)
    worst = float(np.max(err / (4 * EPS32 * mag + 1e-30)))
    announce(f"  update: max |U1 - formula| {err.max():.3e}, worst ratio to the rounding bound {worst:.2f}")
    assert worst <= 1.0


def test_ellipsoid_step_adjoint_128_central_differences():
    announce("full size: 128^3 step adjoint vs central differences")
    sc = scenes.scene_ellipsoid_rollout(seed=1, n=128, steps=1)
    g = Grid(sc.n, sc.dx)
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    th, ct = poses[0], sc.ctrl[0]
    rng = np.random.default_rng(11)
    vdir = scenes.curl_noise(sc.n, sc.dx, rng)
    wdir = rng.standard_normal(g.nfaces)
    h = 1e-3
    with Sim(ellipsoid_cfg(sc.n, tol=1e-7, precision="fp32")) as sim:
        u0 = dev(sc.u0)
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        _, st0 = sim.step(u0, th, ct, p_out=P)
        gu, _ = sim.step_adjoint(u0, dev(wdir), th, ct, p_n1=P)
        up, _ = sim.step(dev(sc.u0 + h * vdir), th, ct)
        um, _ = sim.step(dev(sc.u0 - h * vdir), th, ct)
        torch.cuda.synchronize()
    lhs = float(np.dot(host(gu), vdir))
    fd = float(np.dot(wdir, host(up) - host(um))) / (2 * h)
    rel = abs(lhs - fd) / abs(fd)
    announce(f"  <J^T w, v> {lhs:.6e}  central difference {fd:.6e}  rel {rel:.2e}")
    assert rel <= 5e-3


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_sphere_projection_256_fullsize(precision):
    announce(f"full size: 256^3 twenty-sphere projection, {precision} V-cycle")
    sc = scenes.scene_spheres_projection(seed=0, n=256, count=20)
    g = Grid(sc.n, sc.dx)
    tol = 1e-6
    with Sim(sphere_cfg(sc.n, sc.spheres, tol=tol, precision=precision)) as sim:
        alpha = torch.empty(g.nfaces, dtype=torch.float32, device="cuda")
        sim.set_geometry(sc.spheres.ravel(), alpha_out=alpha)
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u = dev(sc.u0)
        _, st = sim.project(u, sc.spheres.ravel(), p_out=P)
        torch.cuda.synchronize()
    announce(f"  solve: {st}")
    assert st["converged"]
    al, Ph = host(alpha).astype(np.float64), host(P)
    del alpha, P, u
    # FP64 residual of the returned pressure with the oracle's operator on the
    # same fractions (static walls and spheres: U_s = 0); FP32 storage of P adds
    # at most |A| eps |P| with |A| <= 12 (a row sums 2 * 6 fractions <= 1)
    ops = Operators(g, al)
    k = sc.dt / sc.dx
    b = (ops.GT @ (al * sc.u0)) / k
    act = ops.active
    r = np.where(act, b - ops.apply(Ph.astype(np.float64)), 0.0)
    bn = np.linalg.norm(np.where(act, b, 0.0))
    rel = np.linalg.norm(r) / bn
    bound = 1.5 * tol + 12.0 * EPS32 * np.linalg.norm(Ph) / bn
    announce(f"  FP64 relative residual {rel:.3e} (bound {bound:.3e}), CG iterations {st['iters']}")
    assert rel <= bound
