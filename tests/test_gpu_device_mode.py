"""Device solve mode: no call waits on the host, so a whole step can be
captured into a graph.

* A step, its adjoint and a Poisson solve in the device mode equal the
  host-checked mode's bitwise (the same kernels run the same iterations;
  kernels enqueued after convergence exit at once).
* One whole step captured into a graph and replayed several times, with the
  program's own eager work and synchronisations between the replays, equals
  the eager step bitwise on every replay.
* A budget too small to converge is reported in the device-written stats, and
  a pageable host stats pointer is refused before anything is enqueued.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import scenes
from paper_2405_14903_amd import _lib as L
from paper_2405_14903_amd.sim import Sim, ellipsoid_poses
from tests.gpu_common import announce, dev, ellipsoid_cfg, sphere_cfg

pytestmark = pytest.mark.gpu


def _ellipsoid_case(n=32, precision="fp32"):
    sc = scenes.scene_ellipsoid_rollout(seed=2, n=n, steps=2)
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    return sc, poses, ellipsoid_cfg(sc.n, tol=1e-6, precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_device_mode_equals_host_mode(precision):
    announce(f"device solve mode vs host-checked mode, {precision}")
    sc, poses, cfg = _ellipsoid_case(precision=precision)
    out = {}
    for mode in ("host", "device"):
        with Sim(cfg) as sim:
            sim.set_solve_mode(mode, 40)
            u0 = dev(sc.u0)
            P = torch.empty(sim.nc, dtype=torch.float32, device="cuda")
            u1, st = sim.step(u0, poses[0], sc.ctrl[0], p_out=P)
            gbar = dev(np.random.default_rng(1).standard_normal(sim.nf))
            gth = torch.zeros(15, dtype=torch.float64, device="cuda")
            gct = torch.zeros(6, dtype=torch.float64, device="cuda")
            gu, sta = sim.step_adjoint(u0, gbar, poses[0], sc.ctrl[0], p_n1=P, g_theta=gth, g_ctrl=gct)
            x = torch.zeros(sim.nc, dtype=torch.float32, device="cuda")
            b = torch.tensor(np.random.default_rng(2).uniform(-1, 1, sim.nc), dtype=torch.float32, device="cuda")
            b -= b.mean()
            _, sts = sim.poisson_solve(b, x, tol=1e-6)
            torch.cuda.synchronize()
            dct = lambda s: s.as_dict() if hasattr(s, "as_dict") and not isinstance(s, dict) else s  # noqa: E731
            out[mode] = ([t.clone() for t in (u1, P, gu, gth, gct, x)], [dct(s) for s in (st, sta, sts)])
    th, sh = out["host"]
    td, sd = out["device"]
    announce(f"  host stats {sh}")
    announce(f"  device stats {sd}")
    for a, b in zip(th, td):
        assert torch.equal(a, b)
    for a, b in zip(sh, sd):
        assert a["iters"] == b["iters"] and a["converged"] and b["converged"]
        assert a["true_rel_res"] == b["true_rel_res"]


@pytest.mark.parametrize("geom", ["spheres", "ellipsoid"])
def test_whole_step_captured_in_a_graph(geom):
    announce(f"whole step captured into a graph ({geom}), replayed against the eager step")
    if geom == "spheres":
        sc = scenes.scene_sphere_rollout(seed=4, n=32, steps=1)
        cfg = sphere_cfg(sc.n, sc.spheres, tol=1e-6, precision="fp16")
        theta, ctrl = sc.spheres.ravel(), None
    else:
        sc, poses, cfg = _ellipsoid_case(precision="fp16")
        theta, ctrl = poses[1], sc.ctrl[1]
    with Sim(cfg) as sim:
        sim.set_solve_mode("device", 32)
        u0 = dev(sc.u0)
        eager, _ = sim.step(u0, theta, ctrl, stats=False)
        eager = eager.clone()
        u_in = u0.clone()
        u_out = torch.empty_like(u0)
        torch.cuda.synchronize()
        # warm the captured path once on a side stream, as torch recommends
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            sim.step(u_in, theta, ctrl, u_out=u_out, stats=False)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            sim.step(u_in, theta, ctrl, u_out=u_out, stats=False)
        for rep in range(3):
            u_out.fill_(float("nan"))
            u_in.copy_(u0)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            same = torch.equal(u_out, eager)
            announce(f"  replay {rep}: equal to the eager step: {same}")
            assert same
            # eager work between replays: a step of its own on the same handle
            sim.step(u0, theta, ctrl, stats=False)
            torch.cuda.synchronize()


def test_device_mode_budget_and_stats_pointer():
    announce("device mode: unconverged budget in the stats; pageable stats pointer refused")
    sc, poses, cfg = _ellipsoid_case()
    with Sim(cfg) as sim:
        sim.set_solve_mode("device", 2)
        u1, st = sim.step(dev(sc.u0), poses[0], sc.ctrl[0])
        d = st.as_dict()
        announce(f"  budget 2: {d}")
        assert d["iters"] == 2 and not d["converged"] and not d["nonfinite"] and d["rel_res"] > 1e-6
        host_st = L.SimStats()
        u_in = dev(sc.u0)
        u_out = torch.empty_like(u1)
        th = np.ascontiguousarray(poses[0], np.float64)
        ct = np.ascontiguousarray(sc.ctrl[0], np.float64)
        dp = C.POINTER(C.c_double)
        rc = sim.lib.sim_step(sim.h, C.c_void_p(u_in.data_ptr()), th.ctypes.data_as(dp),
                              ct.ctypes.data_as(dp), C.c_void_p(u_out.data_ptr()), None, C.byref(host_st),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert rc == L.SIM_EINVAL
