"""The library's serving pool (sim_pool_*) on the GPU.

* A mix of episodes on two grids (forward + adjoint rollouts, a forward-only
  rollout, a pressure projection) run together through the pool equal the
  same work done one call at a time through the handle API: final velocity,
  loss, dJ/du0 and the per-step shape / control partials.  The second
  episode on a grid runs in the device solve mode with the budget the first
  (host-checked) one set, so both solve modes are covered.
  The units in flight are bounded by grid cells there, so the bound's
  scheduling is covered too.
* Admission: a full pool or budget answers busy; a finished episode's handle
  and buffer are reused by the next episode on its grid, and idle handles
  make room for a new grid.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from paper_2405_14903_amd import _lib as L
from paper_2405_14903_amd.pool import Pool
from paper_2405_14903_amd.rollout import Rollout
from paper_2405_14903_amd.sim import Config, Sim, _host_doubles, ellipsoid_poses, sim_footprint
from tests.gpu_common import announce, dev, host, rel_l2

pytestmark = pytest.mark.gpu

OCTANT = ((0.5, 0.5, 0.5), (1.0, 1.0, 1.0))


def _cfg(n):
    return Config(n=(n, n, n), dx=1.0 / n, dt=0.5 / n, geom="ellipsoid", tol=1e-7, precision="fp16")


def _episode(n, seed, steps):
    sc = scenes.scene_ellipsoid_rollout(seed=seed, n=n, steps=steps)
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    return sc, np.asarray(poses), np.asarray(sc.ctrl)


def _reference_adjoint(cfg, sc, every):
    with Sim(cfg) as sim:
        ro = Rollout.ellipsoid(sim, sc.theta0, sc.ctrl, every=every, warm_start="adjoint")
        uT = ro.forward(dev(sc.u0))
        J, g = sim.loss_box(uT)
        ro.backward(g)
        torch.cuda.synchronize()
        return host(uT), float(J.item()), host(ro.g0), ro.g_steps.cpu().numpy(), ro.g_ctrl_direct.cpu().numpy()


def _reference_forward(cfg, sc, poses):
    with Sim(cfg) as sim:
        u = dev(sc.u0)
        for k in range(len(poses)):
            u, _ = sim.step(u, poses[k], sc.ctrl[k])
        torch.cuda.synchronize()
        return host(u)


def test_pool_mix_equals_one_call_at_a_time():
    announce("serving pool: forward + adjoint, forward-only and projection episodes on 32^3 and 48^3 together")
    T, K = 8, 4
    c32, c48 = _cfg(32), _cfg(48)
    sa, pa, ca = _episode(32, 1, T)
    sb, pb, cb = _episode(48, 2, 6)
    sc_, pc, cc = _episode(32, 3, 1)
    sd, pd, cd = _episode(32, 4, T)
    jobs = [dict(cfg=c32, kind="fwd+adj", u0=dev(sa.u0), theta=pa, ctrl=ca, steps=T, every=K, box=OCTANT),
            dict(cfg=c48, kind="fwd", u0=dev(sb.u0), theta=pb, ctrl=cb, steps=6),
            dict(cfg=c32, kind="poisson", u0=dev(sc_.u0), theta=pc[:1], ctrl=cc[:1]),
            dict(cfg=c32, kind="fwd+adj", u0=dev(sd.u0), theta=pd, ctrl=cd, steps=T, every=K, box=OCTANT)]
    # at most one 48^3 unit's worth of cells in flight: a 48^3 unit runs alone,
    # 32^3 units run side by side
    with Pool(budget_bytes=8 << 30, max_active=4, inflight_cells=48 ** 3) as pool:
        first = pool.run(jobs[:1])            # sets the 32^3 iteration budget (host-checked)
        rest = pool.run(jobs[1:])             # the others together, 32^3 in the device solve mode
    res = first + rest
    for r in res:
        assert r["status"] == 0 and r["worst"]["converged"], r["worst"]
    announce(f"  most CG iterations per episode: {[r['worst']['iters'] for r in res]}")
    for r, sc in ((res[0], sa), (res[3], sd)):
        uT, J, g0, gth, gct = _reference_adjoint(c32, sc, K)
        e = [rel_l2(host(r["u"]), uT), abs(r["J"] - J) / abs(J), rel_l2(host(r["g_u0"]), g0),
             rel_l2(r["g_theta"].cpu().numpy(), gth), rel_l2(r["g_ctrl"].cpu().numpy(), gct)]
        announce("  fwd+adj: u_T {:.1e}, J {:.1e}, dJ/du0 {:.1e}, dJ/dtheta {:.1e}, dJ/dctrl {:.1e}".format(*e))
        assert e[0] <= 1e-6 and e[1] <= 1e-6 and max(e[2:]) <= 1e-5, e
    e = rel_l2(host(res[1]["u"]), _reference_forward(c48, sb, pb))
    announce(f"  fwd 48^3: u_T {e:.1e}")
    assert e <= 1e-6
    with Sim(c32) as sim:
        ref, _ = sim.project(dev(sc_.u0), pc[0], cc[0])
        torch.cuda.synchronize()
    e = rel_l2(host(res[2]["u"]), host(ref))
    announce(f"  projection 32^3: {e:.1e}")
    assert e <= 1e-6


def test_pool_admission_busy_reuse_and_eviction():
    announce("serving pool admission: busy answers, handle reuse, idle eviction")
    c32, c48 = _cfg(32), _cfg(48)
    s32, p32, k32 = _episode(32, 5, 2)
    s48, p48, k48 = _episode(48, 6, 2)
    # room for one 48^3 handle and its episode's few MB, not for a second handle
    budget = sim_footprint(c48) + (4 << 20)
    assert sim_footprint(c32) + (2 << 20) < budget
    job32 = dict(cfg=c32, kind="fwd", u0=dev(s32.u0), theta=p32, ctrl=k32, steps=2)
    job48 = dict(cfg=c48, kind="fwd", u0=dev(s48.u0), theta=p48, ctrl=k48, steps=2)
    with Pool(budget_bytes=budget, max_active=2) as pool:
        a = pool.admit(**job48)
        assert a is not None
        assert pool.admit(**job48) is None     # a second 48^3 handle does not fit
        assert pool.admit(**job32) is None     # nor a 32^3 one while the first is busy
        while pool.tick():
            pass
        ra = pool.result(a)
        b = pool.admit(**job48)                # reuses the idle 48^3 handle
        assert b is not None
        while pool.tick():
            pass
        rb = pool.result(b)
        c = pool.admit(**job32)                # frees the idle 48^3 handle to fit
        assert c is not None
        while pool.tick():
            pass
        rc = pool.result(c)
    assert ra["status"] == 0 and rb["status"] == 0 and rc["status"] == 0
    # the same episode twice on one handle (host-checked, then with the learned
    # budget in the device solve mode): the same result
    np.testing.assert_allclose(host(rb["u"]), host(ra["u"]), rtol=0, atol=1e-6 * float(ra["u"].abs().max()))
    with Pool(budget_bytes=8 << 30, max_active=1) as pool:
        s = pool.admit(**job32)
        assert pool.admit(**job32) is None     # no free slot
        while pool.tick():
            pass
        pool.result(s)


def test_pool_host_checked_episode_and_flags():
    announce("serving pool: an episode admitted host-checked equals the device-mode one; unknown flags rejected")
    c32 = _cfg(32)
    s32, p32, k32 = _episode(32, 7, 4)
    job = dict(cfg=c32, kind="fwd", u0=dev(s32.u0), theta=p32, ctrl=k32, steps=4)
    with Pool(budget_bytes=8 << 30, max_active=2) as pool:
        first = pool.run([job])[0]                       # learns the budget (host-checked)
        a = pool.admit(**job)                            # device mode
        b = pool.admit(**job, host_checked=True)         # host-checked again
        while pool.tick():
            pass
        ra, rb = pool.result(a), pool.result(b)
        # flags other than SIM_EP_HOST_CHECKED are rejected before anything runs
        d = c32.desc()
        ep = L.SimEpisode()
        ep.desc, ep.kind, ep.steps, ep.every, ep.flags = d, L.SIM_EP_FORWARD, 4, 1, 2
        th, thp = _host_doubles(p32, 4 * d.n_params, "theta")
        ct, ctp = _host_doubles(k32, 4 * d.n_ctrl, "ctrl")
        ep.theta, ep.ctrl = thp, ctp
        slot = C.c_int32(-1)
        u0 = dev(s32.u0)
        assert pool.lib.sim_pool_admit(pool.h, C.byref(ep), C.c_void_p(u0.data_ptr()), C.byref(slot)) == L.SIM_EINVAL
    for r in (first, ra, rb):
        assert r["status"] == 0, r["worst"]
    ref = host(first["u"])
    np.testing.assert_allclose(host(ra["u"]), ref, rtol=0, atol=1e-6 * float(np.abs(ref).max()))
    np.testing.assert_allclose(host(rb["u"]), ref, rtol=0, atol=1e-6 * float(np.abs(ref).max()))
