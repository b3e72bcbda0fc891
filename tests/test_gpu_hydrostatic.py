"""Hydrostatic balance on the GPU (a constant body force, this project's
addition for this check; the paper has none): a fluid at rest
around a static sphere under gravity stays at rest, and the pressure is the
discrete linear potential, k (G P) = dt g on every face carrying fluid; the
step matches the oracle's."""
import numpy as np
import pytest
import torch

from oracle.geometry import sphere_geometry
from oracle.mac import Grid
from oracle.projection import Operators
from oracle.step import Step, StepParams
from paper_2405_14903_amd.sim import Config, Sim
from tests.gpu_common import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,precision", [(32, "fp32"), (48, "fp16")])
def test_hydrostatic_balance_gpu(n, precision):
    announce(f"hydrostatic balance {n}^3 {precision}")
    dx = 1.0 / n
    dt = 0.5 * dx
    grav = (0.0, 0.0, -9.8)
    sph = np.array([[0.5, 0.45, 0.55, 0.22]])
    g = Grid((n, n, n), dx)
    geo = sphere_geometry(g, sph)
    cfg = Config(n=(n, n, n), dx=dx, dt=dt, gravity=grav, geom="spheres", n_spheres=1, tol=1e-7,
                 precision=precision, max_iter=200)
    with Sim(cfg) as sim:
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u1, st = sim.step(dev(np.zeros(g.nfaces)), sph.ravel(), p_out=P)
        torch.cuda.synchronize()
    announce(f"  solve: {st}")
    assert st["converged"]
    u1h, Ph = host(u1), host(P)
    scale = dt * 9.8
    k = dt / dx
    # at rest: what is left is the solve's tolerance on dt |g| and the FP32
    # rounding of P (a face difference of two values of size max |P|)
    bound = 1e-5 * scale + 4.0 * float(np.finfo(np.float32).eps) * k * np.abs(Ph).max()
    announce(f"  max |U1| {np.abs(u1h).max():.2e} (bound {bound:.2e}, dt |g| {scale:.3f})")
    assert np.abs(u1h).max() <= bound
    gp = k * (Operators(g, geo.alpha).G @ Ph)
    zf = np.concatenate([np.zeros(g.nf(0) + g.nf(1)), np.ones(g.nf(2))])
    # the update weights k G P by alpha, so the solve pins it on a face only to
    # about its tolerance / alpha: alpha-weighted on every fluid face (what the
    # velocity sees), unweighted where the face is at least a tenth open
    m = geo.alpha > 0
    np.testing.assert_allclose((geo.alpha * gp)[m], (-scale * geo.alpha * zf)[m], rtol=0, atol=bound)
    o = geo.alpha >= 0.1
    np.testing.assert_allclose(gp[o], (-scale * zf)[o], rtol=0, atol=bound)
    st_o = Step(StepParams(g, dt, gravity=grav, tol=1e-12), np.zeros(g.nfaces), geo.alpha, geo.us)
    assert np.abs(u1h - st_o.result).max() <= bound
