"""The allocation-free box loss against the handle's box loss, on two calls in
a row through the C ABI, the second on a smaller grid."""
import numpy as np
import pytest
import torch

import scenes
from paper_2405_14903_amd.sim import Sim, loss_box_noalloc
from tests.gpu_common import announce, dev, sphere_cfg

pytestmark = pytest.mark.gpu


def test_loss_box_noalloc_matches_handle_entry_point():
    for n, lo, hi in ((64, (0.5, 0.5, 0.5), (1.0, 1.0, 1.0)), (24, (0.1, 0.25, 0.0), (0.7, 1.0, 0.5))):
        announce(f"allocation-free box loss, {n}^3")
        dx = 1.0 / n
        u = dev(scenes.curl_noise((n, n, n), dx, np.random.default_rng(n)))
        with Sim(sphere_cfg((n, n, n), np.array([[0.5, 0.5, 0.5, 0.2]]))) as sim:
            J_ref, g_ref = sim.loss_box(u, lo, hi)
            torch.cuda.synchronize()
        J, g = loss_box_noalloc(u, (n, n, n), dx, lo, hi)
        torch.cuda.synchronize()
        announce(f"  J {float(J.item()):.15e} vs {float(J_ref.item()):.15e}")
        # the same kernels over the same partial-sum layout: the same bits
        assert torch.equal(J, J_ref) and torch.equal(g, g_ref)
        assert float(J.item()) > 0.0
