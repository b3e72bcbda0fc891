"""Closed-loop control through the differentiable simulator: a gym-style
environment and a two-layer MLP controller trained by back-propagation
through the rollout (NeuralFluid, Sec. Neural Fluid Control; Sec. Benchmarks
and Applications: controllers are two-layer MLPs whose state holds a temporal
encoding of the step and a flow measurement, trained with gradient clipping
at 1.0).

The scene is the moving-ellipsoid box: the controller sets the body's linear
and angular velocity (6 values in [-0.5, 0.5]) every step, from an
observation of the temporal encoding (sin and cos of the step's phase) and the
kinetic energy of the fluid in the octant [0.5, 1]^3 relative to its initial
value; the task asks that energy to follow a target profile over the episode
(by default falling linearly to 70% of its initial value).  The environment runs on
one library handle (optionally in the device solve mode the serving loop
uses); `train_step` runs one episode forward with the controller in the loop,
then the hand-written adjoint backward, and hands dJ/d(controls) to the MLP's
autograd.  Reading: the observation enters the controller as data (its
gradient w.r.t. the velocity field is not propagated); the paper does not
say whether its controllers differentiate through their observations.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .rollout import Rollout
from .sim import Config, Sim, ellipsoid_poses


class MLPController(torch.nn.Module):
    """obs -> 6 controls in [-limit, limit]: Linear, tanh, Linear, limit * tanh."""

    def __init__(self, obs_dim=3, hidden=64, limit=0.5, seed=0):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        self.l1 = torch.nn.Linear(obs_dim, hidden, dtype=torch.float64)
        self.l2 = torch.nn.Linear(hidden, 6, dtype=torch.float64)
        with torch.no_grad():
            for lin in (self.l1, self.l2):
                lin.weight.copy_(torch.randn(lin.weight.shape, generator=g, dtype=torch.float64)
                                 / math.sqrt(lin.in_features))
                lin.bias.zero_()
        self.limit = limit

    def forward(self, obs):
        return self.limit * torch.tanh(self.l2(torch.tanh(self.l1(obs))))


class FluidControlEnv:
    """Gym-style environment (reset / step) over one simulator handle.

    reset(seed) -> observation; step(action) -> (observation, reward, done,
    info).  The reward is minus the squared miss of the target energy."""

    def __init__(self, n=32, steps=16, profile=None, precision="fp32", device_mode=False, tol=1e-6):
        self.n, self.T = n, steps
        self.cfg = Config(n=(n, n, n), dx=1.0 / n, dt=0.5 / n, geom="ellipsoid", tol=tol, precision=precision)
        self.sim = Sim(self.cfg)
        if device_mode:
            self.sim.set_solve_mode("device", 48)
        # target octant energy after each step, as a fraction of the initial energy
        self.profile = np.asarray(profile if profile is not None else np.linspace(1.0, 0.7, steps + 1)[1:],
                                  np.float64)

    def close(self):
        self.sim.close()

    def _obs(self, n, energy):
        ph = 2.0 * math.pi * n / self.T
        return np.array([math.sin(ph), math.cos(ph), energy / self.e0])

    def reset(self, seed=0):
        import scenes
        sc = scenes.scene_ellipsoid_rollout(seed=seed, n=self.n, steps=self.T)
        self.theta0 = sc.theta0
        self.u = torch.tensor(sc.u0, dtype=torch.float32, device="cuda")
        self.u0 = self.u.clone()
        self.ctrl = np.zeros((0, 6))
        self.n_step = 0
        J, _ = self.sim.loss_box(self.u)
        self.e0 = float(J.item())
        self.target = self.e0 * self.profile
        return self._obs(0, self.e0)

    def step(self, action):
        a = np.clip(np.asarray(action, np.float64).reshape(6), -0.5, 0.5)
        self.ctrl = np.vstack([self.ctrl, a])
        pose = ellipsoid_poses(self.theta0, self.ctrl, self.cfg.dt)[-1]
        self.u, _ = self.sim.step(self.u, pose, a, stats=False)
        J, _ = self.sim.loss_box(self.u)
        e = float(J.item())
        r = -((e - self.target[self.n_step]) / self.e0) ** 2
        self.n_step += 1
        done = self.n_step >= self.T
        return self._obs(self.n_step, e), r, done, {"energy": e}


def episode_loss(env: FluidControlEnv, controller: MLPController, seed=0, every=4, fixed_obs=None):
    """One closed-loop episode: the controller acts on each observation; J =
    sum over steps of ((octant energy - target) / initial energy)^2.  Returns (J, rollout, list
    of the controller's output tensors, observations) with the adjoint
    already run, so dJ/d(controls) is available from the rollout.
    fixed_obs: replay these observations instead of the episode's own (the
    controller then runs open loop; used to check gradients)."""
    sim = env.sim
    obs = env.reset(seed)
    outs, ctrls, seen = [], [], []
    for n in range(env.T):
        if fixed_obs is not None:
            obs = fixed_obs[n]
        seen.append(np.asarray(obs))
        o = torch.tensor(obs, dtype=torch.float64)
        c = controller(o)
        outs.append(c)
        ctrls.append(c.detach().numpy())
        obs, _, _, _ = env.step(ctrls[-1])
    ctrl = np.stack(ctrls)
    target = torch.tensor(env.target, dtype=torch.float64, device="cuda")

    def step_loss(n, u):
        E, gE = sim.loss_box(u)
        miss = (E - target[n]) / env.e0
        return miss * miss, (2.0 * miss / env.e0).float() * gE
    ro = Rollout.ellipsoid(sim, env.theta0, ctrl, every=every)
    ro.step_loss = step_loss
    ro.forward(env.u0)
    ro.backward(torch.zeros_like(env.u0))
    return float(ro.J.item()), ro, outs, seen


def train_step(env: FluidControlEnv, controller: MLPController, optimizer, seed=0, clip=1.0):
    """Forward episode, hand-written adjoint backward, MLP update with the
    gradient norm clipped at `clip`.  Returns (J, gradient norm before clipping)."""
    J, ro, outs, _ = episode_loss(env, controller, seed)
    _, g_ctrl = ro.geometry_gradients()            # dJ/d(controls), (T, 6)
    optimizer.zero_grad()
    torch.autograd.backward(outs, [torch.tensor(g, dtype=torch.float64) for g in g_ctrl])
    gnorm = float(torch.nn.utils.clip_grad_norm_(controller.parameters(), clip))
    optimizer.step()
    return J, gnorm
