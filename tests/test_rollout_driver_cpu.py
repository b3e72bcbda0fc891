"""The BPTT driver (checkpointing, segment recomputation, per-step adjoints,
pose chain) checked on the CPU: a stand-in handle runs the oracle's step and
adjoint, and the driver's gradients must equal the oracle's own BPTT."""
import numpy as np
import pytest
import torch

import scenes
from oracle.mac import Grid
from oracle.geometry import sphere_geometry, EllipsoidGeometry
from oracle.rollout import StaticRollout, EllipsoidRollout, octant_loss
from oracle.step import Step, StepParams
from paper_2405_14903_amd import rollout as R


class OracleHandle:
    """Duck-typed stand-in for Sim running the FP64 oracle on CPU tensors."""

    def __init__(self, prm, kind, spheres=None):
        self.prm, self.kind, self.spheres = prm, kind, spheres
        g = prm.grid
        self.nf, self.nc = g.nfaces, g.ncells
        self.n_params, self.n_ctrl = (15, 6) if kind == "ellipsoid" else (4 * len(spheres), 0)
        self.cfg = type("C", (), {"dt": prm.dt})()
        self.steps_done = 0
        self.replays = 0
        self.pressure_dtype = torch.float64
        self.warm_calls = []

    def set_warm_start(self, pressure=False, adjoint=False):
        # the oracle solves exactly, so warm starts change nothing but the record
        self.warm_calls.append((pressure, adjoint))

    def _geo(self, th, ct):
        g = self.prm.grid
        if self.kind == "ellipsoid":
            th = np.asarray(th)
            return EllipsoidGeometry(g, th[:3], th[3:6], th[6:].reshape(3, 3), ct[:3], ct[3:])
        return sphere_geometry(g, self.spheres)

    def step(self, u, th, ct, u_out=None, p_out=None, stats=False):
        geo = self._geo(th, ct)
        st = Step(self.prm, u.double().numpy(), geo.alpha, geo.us)
        u_out.copy_(torch.from_numpy(st.result))
        if p_out is not None:
            p_out.copy_(torch.from_numpy(st.P))
        self.steps_done += 1
        return u_out, None

    def step_replay(self, u, p, th, ct, u_out=None):
        """The update of Eq. u_next_matrix from the given pressure (the oracle's
        pieces: its advection, G and the face average), no solve."""
        from oracle.advection import Advection, laplacian_faces
        from oracle.projection import Operators
        geo = self._geo(th, ct)
        uh = Advection(self.prm.grid, u.double().numpy(), self.prm.dt).result
        if self.prm.nu:
            uh = uh + self.prm.dt * self.prm.nu * laplacian_faces(self.prm.grid, uh)
        G = Operators(self.prm.grid, geo.alpha).G
        W = uh - self.prm.k * (G @ p.double().numpy())
        u_out.copy_(torch.from_numpy(geo.alpha * W + (1.0 - geo.alpha) * geo.us))
        self.replays += 1
        return u_out

    def step_adjoint(self, u_n, g, th, ct, p_n1=None, g_u_n=None, g_theta=None, g_ctrl=None, stats=False):
        geo = self._geo(th, ct)
        st = Step(self.prm, u_n.double().numpy(), geo.alpha, geo.us)
        gu, galpha, gus = st.vjp(g.double().numpy())
        g_u_n.copy_(torch.from_numpy(gu))
        if self.kind == "ellipsoid" and g_theta is not None:
            d = geo.vjp(galpha, gus)
            g_theta += torch.from_numpy(np.concatenate([d["c"], d["a"], d["R"].ravel()]))
            g_ctrl += torch.from_numpy(np.concatenate([d["v"], d["w"]]))
        return g_u_n, None


@pytest.mark.parametrize("store", [True, False])
@pytest.mark.parametrize("every", [1, 3, "sqrt"])
def test_static_rollout_driver_matches_oracle_bptt(every, store):
    sc = scenes.scene_sphere_rollout(seed=0, n=10, steps=5)
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-12)
    ro_o = StaticRollout(prm, sc.u0, sc.spheres)
    J_o, gT = octant_loss(g, ro_o.forward(5))
    gu_o = ro_o.backward(gT)
    h = OracleHandle(prm, "spheres", sc.spheres)
    ro = R.Rollout(h, 5, lambda n: (sc.spheres.ravel(), None), every=every, store_pressure=store)
    uT = ro.forward(torch.from_numpy(sc.u0.copy()))
    np.testing.assert_allclose(uT.numpy(), ro_o.hist[-1], atol=1e-13)
    gu = ro.backward(torch.from_numpy(gT.copy()))
    np.testing.assert_allclose(gu.numpy(), gu_o, rtol=1e-9, atol=1e-12 * np.abs(gu_o).max())
    # stored pressures: the recomputation replays every step (no solve)
    assert (h.replays == 5) == store and (h.steps_done == 5) == store


def test_ellipsoid_rollout_driver_matches_oracle_bptt():
    sc = scenes.scene_ellipsoid_rollout(seed=1, n=10, steps=4)
    sc.theta0[3:6] = [0.24, 0.2, 0.28]
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-12)
    ro_o = EllipsoidRollout(prm, sc.u0, sc.theta0, sc.ctrl)
    _, gT = octant_loss(g, ro_o.forward())
    gu_o, gth_o, gct_o = ro_o.backward(gT)
    h = OracleHandle(prm, "ellipsoid")
    ro = R.Rollout.ellipsoid(h, sc.theta0, sc.ctrl, every=3)
    ro.forward(torch.from_numpy(sc.u0.copy()))
    gu = ro.backward(torch.from_numpy(gT.copy()))
    gth, gct = ro.geometry_gradients()
    np.testing.assert_allclose(gu.numpy(), gu_o, rtol=1e-9, atol=1e-12 * np.abs(gu_o).max())
    np.testing.assert_allclose(gth, gth_o, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(gct, gct_o, rtol=1e-8, atol=1e-12)


def test_frame_rollout_substeps_and_gradient():
    """CFL frames on the oracle stand-in: sub-step counts from the definition
    (advective and viscous limits) and the driver's gradient against a plain
    chain of the oracle's step adjoints with the same time steps."""
    import math
    sc = scenes.scene_sphere_rollout(seed=2, n=8, steps=3)
    g = Grid(sc.n, sc.dx)
    nu, frame_dt, cfl = 0.02, 2.0 * sc.dx, 0.5
    prm0 = StepParams(g, frame_dt, nu=nu, tol=1e-12)
    h = OracleHandle(prm0, "spheres", sc.spheres)
    h.cfg.dx, h.cfg.nu, h.dt = g.dx, nu, frame_dt

    def set_dt(dt):
        h.prm = StepParams(g, dt, nu=nu, tol=1e-12)
        h.dt = dt
    h.set_dt = set_dt
    h.max_speed = lambda u: float(u.abs().max())
    ro = R.FrameRollout(h, 3, frame_dt, lambda n: (sc.spheres.ravel(), None), every=2, cfl=cfl)
    uT = ro.forward(torch.from_numpy(sc.u0.copy()))
    # the counts from the definition, on the oracle's own states
    geo = sphere_geometry(g, sc.spheres)
    u, us, dts = sc.u0.copy(), [], []
    for m in ro.substeps:
        want = max(1, math.ceil(frame_dt * np.abs(u).max() / (cfl * g.dx) - 1e-12),
                   math.ceil(frame_dt * nu / (g.dx ** 2 / 6.0) - 1e-12))
        assert m == want
        for _ in range(m):
            st = Step(StepParams(g, frame_dt / m, nu=nu, tol=1e-12), u, geo.alpha, geo.us)
            us.append(st)
            dts.append(frame_dt / m)
            u = st.result
    assert ro.dts == dts and sum(ro.substeps) == ro.T > 3
    np.testing.assert_allclose(uT.numpy(), u, atol=1e-12)
    _, gT = octant_loss(g, u)
    gu = ro.backward(torch.from_numpy(gT.copy()))
    gref = gT
    for st in reversed(us):
        gref = st.vjp(gref)[0]
    np.testing.assert_allclose(gu.numpy(), gref, rtol=1e-9, atol=1e-12 * np.abs(gref).max())


@pytest.mark.parametrize("warm", ["adjoint", "all"])
def test_warm_start_passes_reset_and_restore_the_handle(warm):
    """Each pass turns the handle's warm starts on (which also forgets the held
    pressures, so every pass starts its chain from zero) and off at its end;
    forward warm starts refuse a rollout that would re-solve its segments."""
    sc = scenes.scene_sphere_rollout(seed=0, n=8, steps=3)
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-12)
    h = OracleHandle(prm, "spheres", sc.spheres)
    ro = R.Rollout(h, 3, lambda n: (sc.spheres.ravel(), None), every=2, warm_start=warm)
    ro.forward(torch.from_numpy(sc.u0.copy()))
    assert h.warm_calls == [(warm == "all", False), (False, False)]
    ro.backward(torch.zeros(g.nfaces, dtype=torch.float64))
    assert h.warm_calls[2:] == [(False, True), (False, False)]
    with pytest.raises(ValueError):
        R.Rollout(h, 3, lambda n: (sc.spheres.ravel(), None), warm_start="all", store_pressure=False)
    with pytest.raises(ValueError):
        R.Rollout(h, 3, lambda n: (sc.spheres.ravel(), None), warm_start=True)
