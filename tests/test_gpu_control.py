"""Closed-loop control through the simulator: the gym-style environment, the
two-layer MLP controller's gradient from the hand-written adjoint against
central differences (observations held fixed, the reading the controller is
trained under), and a few clipped training steps lowering the loss."""
import numpy as np
import pytest
import torch

from paper_2405_14903_amd.control import FluidControlEnv, MLPController, episode_loss, train_step
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def test_environment_api():
    announce("control environment: reset / step")
    env = FluidControlEnv(n=16, steps=4)
    try:
        obs = env.reset(seed=1)
        assert obs.shape == (3,)
        total = 0.0
        for n in range(4):
            obs, r, done, info = env.step(np.full(6, 0.1))
            total += r
            assert done == (n == 3) and r <= 0.0 and info["energy"] > 0.0
        assert np.isfinite(total)
    finally:
        env.close()


def test_controller_gradient_matches_central_differences():
    announce("controller gradient (adjoint) against central differences")
    env = FluidControlEnv(n=16, steps=6, tol=1e-8)
    try:
        ctl = MLPController(seed=3)
        J, ro, outs, seen = episode_loss(env, ctl, seed=2)
        _, g_ctrl = ro.geometry_gradients()
        ctl.zero_grad()
        torch.autograd.backward(outs, [torch.tensor(g, dtype=torch.float64) for g in g_ctrl])
        params = [(ctl.l2.bias, 0), (ctl.l2.weight, (3, 5)), (ctl.l1.weight, (7, 2))]
        for p, idx in params:
            ad = float(p.grad[idx])
            h = 1e-3
            with torch.no_grad():
                p[idx] += h
            Jp = episode_loss(env, ctl, seed=2, fixed_obs=seen)[0]
            with torch.no_grad():
                p[idx] -= 2 * h
            Jm = episode_loss(env, ctl, seed=2, fixed_obs=seen)[0]
            with torch.no_grad():
                p[idx] += h
            fd = (Jp - Jm) / (2 * h)
            announce(f"  {tuple(p.shape)}{idx}: adjoint {ad:.6e}, central difference {fd:.6e}")
            # central differences straddle the marching-squares kinks of the moving body
            assert abs(ad - fd) <= 5e-2 * max(abs(fd), 1e-2 * abs(J)), (ad, fd)
    finally:
        env.close()


def test_training_lowers_the_loss():
    announce("closed-loop training, gradient clipping 1.0")
    env = FluidControlEnv(n=16, steps=8)
    try:
        ctl = MLPController(seed=0)
        opt = torch.optim.Adam(ctl.parameters(), lr=0.01)
        losses = []
        for it in range(6):
            J, gn = train_step(env, ctl, opt, seed=0)
            losses.append(J)
            announce(f"  iteration {it}: J {J:.4f}, gradient norm {gn:.3e}")
        assert losses[-1] < losses[0], losses
    finally:
        env.close()
