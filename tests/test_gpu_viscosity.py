"""Viscosity (Eq. viscosity_matrix, explicit) and CFL frames on the GPU.

* A viscous step with a static sphere and its adjoint against the oracle's.
* The 2D Taylor-Green vortex in the closed box [0, pi]^3 (an exact solution
  there: it crosses no wall, and its tangential components have zero normal
  derivative) advanced in CFL frames: the decay matches exp(-2 nu t) with an
  error that falls about first order from 32^3 to 64^3 to 128^3, and the 32^3
  run equals the oracle's run of the same sub-steps.
* A frame rollout's gradient w.r.t. the initial velocity against a chain of
  the oracle's step adjoints with the oracle's own sub-step counts.
"""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle.geometry import apply_domain_sides, no_solid_geometry, sphere_geometry
from oracle.mac import Grid
from oracle.rollout import octant_loss
from oracle.step import Step, StepParams
from paper_2405_14903_amd.rollout import FrameRollout
from paper_2405_14903_amd.sim import Config, Sim
from tests.gpu_common import announce, dev, host, rel_l2, sphere_cfg

pytestmark = pytest.mark.gpu


def _substeps(frame_dt, vmax, dx, cfl, nu):
    """The sub-step count from its definition (advective and explicit viscous limits)."""
    return max(1, math.ceil(frame_dt * vmax / (cfl * dx) - 1e-12), math.ceil(frame_dt * nu / (dx * dx / 6.0) - 1e-12))


def test_viscous_step_and_adjoint_parity_32():
    announce("viscous step and adjoint, 32^3 with a sphere, against the oracle")
    sc = scenes.scene_sphere_rollout(seed=1, n=32, steps=1)
    nu = 0.01                               # nu dt / dx^2 = 0.16
    g = Grid(sc.n, sc.dx)
    geo = sphere_geometry(g, sc.spheres)
    ref = Step(StepParams(g, sc.dt, nu=nu, tol=1e-12), sc.u0, geo.alpha, geo.us)
    gbar = np.random.default_rng(3).standard_normal(g.nfaces)
    gref, _, _ = ref.vjp(gbar)
    cfg = sphere_cfg(sc.n, sc.spheres, tol=1e-7)
    cfg.nu = nu
    with Sim(cfg) as sim:
        u0 = dev(sc.u0)
        P = torch.empty(sim.nc, dtype=torch.float32, device="cuda")
        u1, st = sim.step(u0, sc.spheres.ravel(), p_out=P)
        gu, _ = sim.step_adjoint(u0, dev(gbar), sc.spheres.ravel(), p_n1=P)
        torch.cuda.synchronize()
    ef, eb = rel_l2(host(u1), ref.result), rel_l2(host(gu), gref)
    announce(f"  forward rel-L2 {ef:.2e} ({st['iters']} CG iterations), adjoint rel-L2 {eb:.2e}")
    assert ef <= 1e-5 and eb <= 1e-4, (ef, eb)


def _tg_field(g):
    x = [g.face_positions(d) for d in range(3)]
    return np.concatenate([np.sin(x[0][:, 0]) * np.cos(x[0][:, 1]),
                           -np.cos(x[1][:, 0]) * np.sin(x[1][:, 1]),
                           np.zeros(g.nf(2))])


def _tg_gpu(n, nu, t_end, cfl=0.5):
    g = Grid((n, n, n), math.pi / n)
    u0 = _tg_field(g)
    frame_dt = 0.5 * g.dx
    frames = int(round(t_end / frame_dt))
    cfg = Config(n=(n, n, n), dx=g.dx, dt=frame_dt, nu=nu, tol=1e-7, max_iter=300)
    with Sim(cfg) as sim:
        ro = FrameRollout(sim, frames, frame_dt, lambda k: (None, None), every=1 << 30, cfl=cfl,
                          store_pressure=False)
        uT = ro.forward(dev(u0))
        torch.cuda.synchronize()
        out = host(uT)
    return g, u0, out, frames * frame_dt, ro.substeps


def test_taylor_green_closed_box_decay_and_convergence():
    nu, t_end = 0.05, 0.4
    errs, amps = [], []
    for n in (32, 64, 128):
        announce(f"Taylor-Green in the closed box, {n}^3, nu {nu}, CFL frames to t = {t_end}")
        g, u0, uT, t, subs = _tg_gpu(n, nu, t_end)
        exact = u0 * math.exp(-2 * nu * t)
        e = rel_l2(uT, exact)
        amp = (uT @ u0) / (u0 @ u0)
        errs.append(e)
        amps.append(abs(amp - math.exp(-2 * nu * t)))
        announce(f"  {len(subs)} frames, sub-steps {sorted(set(subs))}; field rel-L2 {e:.3e}, amplitude "
                 f"{amp:.6f} vs exp(-2 nu t) {math.exp(-2 * nu * t):.6f}")
    assert errs[1] < 0.65 * errs[0] and errs[2] < 0.65 * errs[1], errs
    assert amps[2] < amps[1] < amps[0], amps
    assert errs[2] < 0.02


def test_taylor_green_32_matches_oracle_substeps():
    nu, t_end, cfl = 0.05, 0.4, 0.5
    announce("Taylor-Green 32^3: GPU frames against the oracle's own sub-steps")
    g, u0, uT, t, subs = _tg_gpu(32, nu, t_end, cfl)
    geo = no_solid_geometry(g)
    geo.alpha, geo.us, geo.fixed = apply_domain_sides(g, np.ones(g.nfaces), np.zeros(g.nfaces))
    frame_dt = 0.5 * g.dx
    u = u0
    oracle_subs = []
    for _ in range(len(subs)):
        m = _substeps(frame_dt, np.abs(u).max(), g.dx, cfl, nu)
        oracle_subs.append(m)
        for _ in range(m):
            u = Step(StepParams(g, frame_dt / m, nu=nu, tol=1e-11), u, geo.alpha, geo.us).result
    e = rel_l2(uT, u)
    announce(f"  sub-steps GPU {subs[:4]}... oracle {oracle_subs[:4]}...; rel-L2 {e:.2e}")
    assert subs == oracle_subs
    assert e <= 1e-5, e


def test_frame_rollout_gradient_vs_oracle():
    announce("CFL frame rollout with viscosity, 16^3 sphere: dJ/du0 against the oracle")
    sc = scenes.scene_sphere_rollout(seed=2, n=16, steps=1)
    nu, frame_dt, cfl, frames = 0.02, 2.0 * sc.dx, 0.5, 3
    g = Grid(sc.n, sc.dx)
    geo = sphere_geometry(g, sc.spheres)
    cfg = sphere_cfg(sc.n, sc.spheres, tol=1e-8)
    cfg.nu, cfg.dt = nu, frame_dt
    with Sim(cfg) as sim:
        ro = FrameRollout(sim, frames, frame_dt, lambda k: (sc.spheres.ravel(), None), every=2, cfl=cfl)
        uT = ro.forward(dev(sc.u0))
        J_o, gT = octant_loss(g, host(uT))
        gu = ro.backward(dev(gT))
        torch.cuda.synchronize()
    steps, u, subs = [], sc.u0, []
    for _ in range(frames):
        m = _substeps(frame_dt, np.abs(u).max(), g.dx, cfl, nu)
        subs.append(m)
        for _ in range(m):
            st = Step(StepParams(g, frame_dt / m, nu=nu, tol=1e-12), u, geo.alpha, geo.us)
            steps.append(st)
            u = st.result
    gref = octant_loss(g, u)[1]
    for st in reversed(steps):
        gref = st.vjp(gref)[0]
    e_u, e_g = rel_l2(host(uT), u), rel_l2(host(gu), gref)
    announce(f"  sub-steps {ro.substeps} (oracle {subs}); u_T rel-L2 {e_u:.2e}; dJ/du0 rel-L2 {e_g:.2e}")
    assert ro.substeps == subs
    assert e_u <= 1e-5 and e_g <= 1e-4, (e_u, e_g)
