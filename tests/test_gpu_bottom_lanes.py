"""The one-workgroup bottom of the V-cycle with one lane per cell against the
generic bottom (NF_MG_BOTTOM_LANES=0).  Both run the same sweeps and
transfers; only the order of the restriction's 8-term sums differs, so the
CG solves take the same number of iterations (within one) and agree to the
solve tolerance.  Grids whose bottoms hold one level (over 64 cells: the
block-wide coarsest sweeps), two levels (a one-wavefront coarsest) and three
levels, a grid that is its own bottom, and a non-cubic chain."""
import os

import numpy as np
import pytest
import torch

import scenes
from paper_2405_14903_amd.sim import Sim, ellipsoid_poses
from tests.gpu_common import announce, dev, ellipsoid_cfg

pytestmark = pytest.mark.gpu


def _run(n3, precision, lanes):
    if not lanes:
        os.environ["NF_MG_BOTTOM_LANES"] = "0"
    try:
        sc = scenes.scene_ellipsoid_rollout(seed=5, n=16, steps=2)   # shape and controls do not depend on n
        dx = 1.0 / n3[0]
        poses = ellipsoid_poses(sc.theta0, sc.ctrl, 0.5 * dx)
        u0 = scenes.curl_noise(n3, dx, np.random.default_rng(5))
        with Sim(ellipsoid_cfg(n3, tol=1e-6, precision=precision)) as sim:
            u = dev(u0)
            outs, iters = [], []
            for s in range(2):
                u, st = sim.step(u, poses[s], sc.ctrl[s])
                assert st["converged"], st
                outs.append(u.clone())
                iters.append(st["iters"])
            # a random seed gradient: with a constant one the result nearly
            # cancels and what is left is the solves' tolerance-level noise
            gbar = dev(np.random.default_rng(6).standard_normal(u.numel()))
            g, sta = sim.step_adjoint(outs[0], gbar, poses[1], sc.ctrl[1])
            iters.append(sta["iters"])
            torch.cuda.synchronize()
            return [o.cpu().double() for o in outs], g.cpu().double(), iters
    finally:
        os.environ.pop("NF_MG_BOTTOM_LANES", None)


@pytest.mark.parametrize("n3,precision", [((64, 64, 64), "fp32"), ((64, 64, 64), "fp16"), ((48, 48, 48), "fp32"),
                                          ((40, 24, 56), "fp32"), ((8, 8, 8), "fp32"), ((16, 32, 64), "fp16")])
def test_lane_bottom_matches_generic_bottom(n3, precision):
    announce(f"bottom lanes vs generic n={n3} {precision}")
    ref, gref, it_ref = _run(n3, precision, False)
    got, g, it = _run(n3, precision, True)
    announce(f"  CG iterations generic {it_ref} lanes {it}")
    assert all(abs(a - b) <= 1 for a, b in zip(it, it_ref))
    for a, b in zip(ref, got):
        assert torch.isfinite(b).all()
        e = float((a - b).norm() / a.norm())
        announce(f"  velocity rel diff {e:.2e}")
        assert e <= 1e-5
    assert torch.isfinite(g).all()
    e = float((g - gref).norm() / gref.norm())
    announce(f"  adjoint rel diff {e:.2e}")
    assert e <= 1e-5
