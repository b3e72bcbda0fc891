"""Differentiable rollouts: back-propagation through time with step checkpointing.

NeuralFluid, Sec. Back-propagation through Time: the per-step adjoint runs in
reverse order over the whole sequence; Sec. Back-propagation through Geometry:
shape and control gradients are accumulated along the way.  Memory is kept
bounded by storing the velocity only every ``every`` steps (``"sqrt"``:
ceil(sqrt(T))) and recomputing each segment's forward before walking it
backwards; the forward is deterministic (fixed-order reductions, zero initial
pressure guess), so the recomputed states equal the original ones bitwise.
By default the first forward also keeps every step's pressure (one cell array
per step, a sixth of a velocity field), and the recomputation replays each
step from it (advection and update, no Poisson solve: the same bits).  The
adjoint pressure solve does not depend on the forward solver's iterates (only
on the converged operator), so no solver state is stored; the adjoint of the
face-average update needs each step's pressure on cut faces.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .sim import Sim, ellipsoid_poses, ellipsoid_poses_adjoint


def checkpoint_stride(T: int, every) -> int:
    if every == "sqrt":
        return max(1, math.ceil(math.sqrt(T)))
    return max(1, int(every))


class Rollout:
    """Forward + adjoint of T steps of one handle.

    ``schedule(n)`` returns the host (theta, ctrl) arrays of step n; for the
    ellipsoid use :meth:`ellipsoid`.
    """

    def __init__(self, sim: Sim, T: int, schedule, every=8, grad_geometry=False, timer=None, step_loss=None,
                 store_pressure=True, warm_start=False):
        self.sim, self.T, self.schedule = sim, int(T), schedule
        self.store_pressure = store_pressure
        # warm_start: False, "adjoint" (each adjoint solve starts from the
        # previous adjoint pressure) or "all" (the forward solves too, from
        # the previous step's pressure).  The handle forgets the held
        # pressures at the start of each pass, so the passes are
        # deterministic; with forward warm starts the recomputation must
        # replay the stored pressures (re-solving would not retrace the
        # first pass).
        if warm_start not in (False, "adjoint", "all"):
            raise ValueError(f"warm_start must be False, 'adjoint' or 'all', not {warm_start!r}")
        if warm_start == "all" and not store_pressure:
            raise ValueError("warm-started forward solves need the stored pressures (store_pressure=True)")
        self.warm_start = warm_start
        self.K = checkpoint_stride(self.T, every)
        self.grad_geometry = grad_geometry
        self.timer = timer
        # CG iterations of every forward and adjoint solve (host solve mode:
        # the report costs nothing more there)
        self.iters = {"fwd": [], "adj": []}
        self.collect = not getattr(sim, "device_mode", False)
        # device solve mode: the solver reports written on the device, kept
        # here when a list is given (the caller reads them after the work)
        self.device_stats = None
        # step_loss(n, u_next) -> (J_n: device double (1,), dJ_n/du_next): a loss
        # on every step's result, summed over the rollout
        self.step_loss = step_loss

    @staticmethod
    def ellipsoid(sim: Sim, theta0, ctrl, every=8, timer=None, store_pressure=True, warm_start=False):
        ctrl = np.asarray(ctrl, np.float64).reshape(-1, 6)
        poses = ellipsoid_poses(theta0, ctrl, sim.cfg.dt)
        ro = Rollout(sim, ctrl.shape[0], lambda n: (poses[n], ctrl[n]), every, grad_geometry=True, timer=timer,
                     store_pressure=store_pressure, warm_start=warm_start)
        ro.theta0 = np.asarray(theta0, np.float64).ravel()
        ro.ctrl = ctrl
        return ro

    def _set_dt(self, n):
        """Per-step time step (CFL sub-stepping): set the handle's dt when it changes."""
        dts = getattr(self, "dts", None)
        if dts is not None and self.sim.dt != dts[n]:
            self.sim.set_dt(dts[n])

    def _step(self, n, u, out, p=None):
        self._set_dt(n)
        th, ct = self.schedule(n)
        if self.timer:
            self.timer.begin("fwd")
        _, st = self.sim.step(u, th, ct, u_out=out, p_out=p, stats=self.collect or self.device_stats is not None)
        if self.timer:
            self.timer.end("fwd")
        self._record(st, "fwd")

    def _record(self, st, kind):
        if st is None:
            return
        if self.device_stats is not None and not isinstance(st, dict):
            self.device_stats.append((kind, st))       # read once the work is done
        else:
            self.iters[kind].append(st["iters"])

    @staticmethod
    def channel(sim: Sim, knots, f, amp, T, every="sqrt", window=None, timer=None, store_pressure=True):
        """The B-spline wall channel: the wall at t = (n + 1) dt in step n, and
        the time-integrated outflow flux sum_n dt dx^2 sum_outlet w U^{n+1}
        (window w: device float32 over the nx * ny outlet faces, or None)."""
        knots = np.ascontiguousarray(knots, np.float64).ravel()
        dt, dx = sim.cfg.dt, sim.cfg.dx
        ctrl = [np.array([(n + 1) * dt, f, amp], np.float64) for n in range(T)]
        loss = lambda n, u: sim.loss_outlet(u, dt * dx * dx, window)   # noqa: E731
        ro = Rollout(sim, T, lambda n: (knots, ctrl[n]), every, grad_geometry=True, timer=timer, step_loss=loss,
                     store_pressure=store_pressure)
        return ro

    def forward(self, u0: torch.Tensor) -> torch.Tensor:
        for _ in self.forward_steps(u0):
            pass
        return self.uT

    def forward_steps(self, u0: torch.Tensor):
        """The forward rollout as a generator: each step is enqueued on the
        current stream, then the generator yields (the serving loop
        interleaves the steps of many episodes).  The result is ``self.uT``."""
        self.ckpt = {0: u0.detach().clone()}
        a = u0.detach().clone()
        b = torch.empty_like(a)
        self.J = torch.zeros(1, dtype=torch.float64, device=u0.device) if self.step_loss else None
        self.P = torch.empty((self.T, self.sim.nc), dtype=getattr(self.sim, "pressure_dtype", torch.float32),
                             device=u0.device) if self.store_pressure else None
        if self.warm_start:
            self.sim.set_warm_start(pressure=self.warm_start == "all")
        for n in range(self.T):
            self._step(n, a, b, self.P[n] if self.P is not None else None)
            a, b = b, a
            if self.step_loss:
                self.J += self.step_loss(n, a)[0]
            if (n + 1) % self.K == 0 and n + 1 < self.T:
                self.ckpt[n + 1] = a.clone()
            self.uT = a
            yield "fwd"
        if self.warm_start:
            self.sim.set_warm_start()
        self.uT = a

    def backward(self, gT: torch.Tensor):
        for _ in self.backward_steps(gT):
            pass
        return self.g0

    def backward_steps(self, gT: torch.Tensor):
        """The adjoint as a generator: yields after each recomputed forward
        step ("fwd") and each adjoint step ("adj").  dJ/du0 is ``self.g0``."""
        sim, T, K = self.sim, self.T, self.K
        dev = gT.device
        g = gT.detach().clone().contiguous()
        gprev = torch.empty_like(g)
        g_steps = torch.zeros((T, sim.n_params), dtype=torch.float64, device=dev) if self.grad_geometry else None
        g_ctrl = torch.zeros((T, sim.n_ctrl), dtype=torch.float64, device=dev) if self.grad_geometry else None
        self.g_steps, self.g_ctrl_direct = g_steps, g_ctrl
        seg_starts = list(range(0, T, K))
        states = [torch.empty_like(g) for _ in range(K + 1)]
        stored = getattr(self, "P", None) is not None
        press = None if stored else [torch.empty(sim.nc, dtype=torch.float32, device=dev) for _ in range(K)]
        if self.warm_start:
            sim.set_warm_start(adjoint=True)
        for s in reversed(seg_starts):
            e = min(s + K, T)
            states[0].copy_(self.ckpt[s])
            for n in range(s, e):
                if stored:
                    self._set_dt(n)
                    th, ct = self.schedule(n)
                    if self.timer:
                        self.timer.begin("replay")
                    sim.step_replay(states[n - s], self.P[n], th, ct, u_out=states[n - s + 1])
                    if self.timer:
                        self.timer.end("replay")
                else:
                    self._step(n, states[n - s], states[n - s + 1], press[n - s])
                yield "fwd"
            for n in range(e - 1, s - 1, -1):
                self._set_dt(n)
                th, ct = self.schedule(n)
                if self.step_loss:
                    g += self.step_loss(n, states[n - s + 1])[1]
                if self.timer:
                    self.timer.begin("adj")
                _, st = sim.step_adjoint(states[n - s], g, th, ct, p_n1=self.P[n] if stored else press[n - s],
                                         g_u_n=gprev,
                                         g_theta=g_steps[n] if g_steps is not None else None,
                                         g_ctrl=g_ctrl[n] if g_ctrl is not None else None,
                                         stats=self.collect or self.device_stats is not None)
                if self.timer:
                    self.timer.end("adj")
                self._record(st, "adj")
                g, gprev = gprev, g
                self.g0 = g
                yield "adj"
        if self.warm_start:
            sim.set_warm_start()
        self.g0 = g

    def geometry_gradients(self):
        """(dJ/dtheta0 (9,), dJ/dctrl (T, 6)) after :meth:`backward` of an ellipsoid rollout."""
        gs = self.g_steps.cpu().numpy()
        gd = self.g_ctrl_direct.cpu().numpy()
        return ellipsoid_poses_adjoint(self.theta0, self.ctrl, self.sim.cfg.dt, gs, gd)


def cfl_substeps(frame_dt, vmax, dx, cfl=0.5, nu=0.0, visc_limit=1.0 / 6.0):
    """Steps a frame of length frame_dt is split into (the paper advances a
    frame by as many solver steps as the CFL condition needs): the smallest m
    with (frame_dt / m) vmax <= cfl dx and, with viscosity, the explicit
    limit nu (frame_dt / m) / dx^2 <= visc_limit."""
    m = 1
    if vmax > 0.0:
        m = max(m, math.ceil(frame_dt * vmax / (cfl * dx) - 1e-12))
    if nu > 0.0:
        m = max(m, math.ceil(frame_dt * nu / (visc_limit * dx * dx) - 1e-12))
    return m


class FrameRollout(Rollout):
    """A rollout of `frames` frames of length frame_dt, each split into CFL
    sub-steps decided from the largest face speed at the frame's start (the
    sub-step counts are piecewise constant in the inputs: no gradient flows
    through them).  The geometry is static (schedule(n) gives the same theta
    for every step); checkpoints every `every` steps (an integer)."""

    def __init__(self, sim: Sim, frames: int, frame_dt: float, schedule, every=8, cfl=0.5, **kw):
        super().__init__(sim, 0, schedule, every, **kw)
        self.frames, self.frame_dt, self.cfl = int(frames), float(frame_dt), float(cfl)

    def forward_steps(self, u0: torch.Tensor):
        sim = self.sim
        self.ckpt = {0: u0.detach().clone()}
        a = u0.detach().clone()
        b = torch.empty_like(a)
        self.J = torch.zeros(1, dtype=torch.float64, device=u0.device) if self.step_loss else None
        self.dts, self.substeps, press = [], [], []
        n = 0
        for _ in range(self.frames):
            m = cfl_substeps(self.frame_dt, sim.max_speed(a), sim.cfg.dx, self.cfl, sim.cfg.nu)
            self.substeps.append(m)
            for _ in range(m):
                self.dts.append(self.frame_dt / m)
                p = torch.empty(sim.nc, dtype=getattr(sim, "pressure_dtype", torch.float32),
                                device=u0.device) if self.store_pressure else None
                press.append(p)
                self._step(n, a, b, p)
                a, b = b, a
                if self.step_loss:
                    self.J += self.step_loss(n, a)[0]
                n += 1
                if n % self.K == 0:
                    self.ckpt[n] = a.clone()
                self.uT = a
                yield "fwd"
        self.T = n
        self.P = torch.stack(press) if self.store_pressure and press else None
        self.uT = a


class ChannelRolloutFn(torch.autograd.Function):
    """J = time-integrated outflow flux of the B-spline wall channel, as a
    torch.autograd.Function of (u0, knots); checkpoints every ceil(sqrt(T))
    steps by default.  u0: device float32; knots: CPU float64
    (SIM_WALL_KNOTS_Y x SIM_WALL_KNOTS_Z)."""

    @staticmethod
    def forward(ctx, u0, knots, sim: Sim, f, amp, T, every="sqrt", window=None):
        ro = Rollout.channel(sim, knots.detach().cpu().numpy(), f, amp, T, every, window)
        ro.forward(u0)
        ctx.ro = ro
        ctx.kshape, ctx.kdev = knots.shape, knots.device
        return ro.J.clone()

    @staticmethod
    def backward(ctx, gJ):
        ro = ctx.ro
        s = float(gJ.reshape(-1)[0])
        g0 = ro.backward(torch.zeros_like(ro.ckpt[0]))
        gk = ro.g_steps.sum(dim=0).cpu().reshape(ctx.kshape)
        return s * g0, (s * gk).to(ctx.kdev), None, None, None, None, None, None


class EllipsoidRolloutFn(torch.autograd.Function):
    """u_T = rollout(u_0, theta_0, ctrl) as a torch.autograd.Function.

    u0: device float32 velocity; theta0 (9,) and ctrl (T, 6): CPU float64.
    Backward runs the hand-written adjoint kernels with checkpointing.
    """

    @staticmethod
    def forward(ctx, u0, theta0, ctrl, sim: Sim, every=8):
        ro = Rollout.ellipsoid(sim, theta0.detach().cpu().numpy(), ctrl.detach().cpu().numpy(), every)
        uT = ro.forward(u0)
        ctx.ro = ro
        ctx.theta_dev = theta0.device
        return uT

    @staticmethod
    def backward(ctx, gT):
        ro = ctx.ro
        g0 = ro.backward(gT.contiguous())
        gth, gct = ro.geometry_gradients()
        return (g0, torch.from_numpy(gth).to(ctx.theta_dev), torch.from_numpy(gct).to(ctx.theta_dev), None, None)


class StaticRolloutFn(torch.autograd.Function):
    """u_T = rollout(u_0) with a static solid (theta fixed); gradient w.r.t. u_0."""

    @staticmethod
    def forward(ctx, u0, sim: Sim, T: int, theta=None, every=8):
        ro = Rollout(sim, T, lambda n: (theta, None), every)
        uT = ro.forward(u0)
        ctx.ro = ro
        return uT

    @staticmethod
    def backward(ctx, gT):
        return ctx.ro.backward(gT.contiguous()), None, None, None, None
