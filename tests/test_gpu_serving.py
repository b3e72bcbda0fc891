"""Serving: continuous batching over device-mode handles gives each request the
same result alone and in the mix (forward bitwise: deterministic kernels, and
device-mode solves run the host-checked solves' iterations; adjoint to the
float-atomic rounding of the advection scatter)."""
import numpy as np
import pytest
import torch

from paper_2405_14903_amd.serving import Request, serve, serve_serial, handle_config, run_episode
from paper_2405_14903_amd.sim import Sim
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def _stream():
    reqs = []
    spec = [(32, 6, "fwd+adj"), (48, 5, "fwd"), (16, 8, "fwd+adj"), (32, 4, "poisson"), (64, 3, "fwd"),
            (16, 5, "fwd+adj"), (48, 4, "fwd+adj"), (32, 7, "fwd")]
    for i, (n, s, m) in enumerate(spec):
        reqs.append(Request(i, 0.01 * i, n, s, m, 1000 + i))
    return reqs


def test_alone_equals_in_the_mix():
    announce("serving alone vs mix")
    mix = _stream()
    summary = serve(mix, budget_bytes=8 << 30, precision="fp32", max_active=6, realtime=True)
    announce(f"  {summary}")
    assert summary["completed"] == len(mix), [r.error for r in mix]
    alone = _stream()
    stream = torch.cuda.Stream()
    for r in alone:
        with Sim(handle_config(r.n, "fp32")) as sim:
            run_episode(sim, r, stream)
    torch.cuda.synchronize()
    for a, b in zip(alone, mix):
        assert not a.error, a.error
        assert torch.equal(a.result["u"], b.result["u"]), a.rid
        assert len(b.step_ms) == (1 if a.mode == "poisson" else a.steps * (1 if a.mode == "fwd" else 3))
        if a.mode == "fwd+adj":
            ga, gb = a.result["g_u0"], b.result["g_u0"]
            e = float((ga - gb).norm() / ga.norm())
            assert e <= 1e-5, (a.rid, e)
            np.testing.assert_allclose(a.result["g_theta0"], b.result["g_theta0"], rtol=1e-4, atol=1e-9)


def test_serial_baseline_waits_for_arrivals():
    announce("serial baseline follows the arrival schedule")
    reqs = [Request(i, 0.2 * i, 16, 3, "fwd", 50 + i) for i in range(3)]
    s = serve_serial(reqs, precision="fp32")
    assert s["completed"] == 3
    for r in reqs:
        assert r.admitted >= r.arrival and r.finished >= r.admitted


def test_budget_rejects_oversized_request():
    announce("serving budget")
    reqs = [Request(0, 0.0, 16, 3, "fwd", 1), Request(1, 0.0, 128, 3, "fwd", 2)]
    s = serve(reqs, budget_bytes=64 << 20, precision="fp32", max_active=2)
    assert s["completed"] == 1 and s["rejected"] == 1
