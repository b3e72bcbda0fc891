"""Parity at the operating points where throughput is measured.

* The benchmark step: the 128^3 moving-ellipsoid step at the benchmark's CG
  tolerance, in FP32 and with the FP16 and BF16 multigrid preconditioners,
  against the oracle's step (its own geometry, advection and an FP64 solve to
  1e-10): velocity relative L2 within the per-step bar 1e-5.
* The differentiable-rollout configuration's 32^3 copy at its real length
  (64 steps, checkpoints every 8): shape and control gradients against the
  oracle's adjoint (1e-3), and against central differences (h = 1e-3).
* The precision configuration (one projection of the twenty-sphere scene) at
  128^3, where the FP64 oracle solves the whole system in a test: pressure
  gradient and projected velocity of the FP32, FP16 and BF16 forms against the
  oracle's solve.
* The octant loss and its seed against the oracle's.
* A closed box with eight floating fluid pockets against the oracle.

Every oracle input is the oracle's own (poses from its pose dynamics, face
fractions from its geometry); nothing computed on the GPU enters it.
"""
import numpy as np
import pytest
import torch

import scenes
from oracle.geometry import EllipsoidGeometry, sphere_geometry
from oracle.mac import Grid
from oracle.projection import Operators, Projection
from oracle.rollout import EllipsoidRollout, octant_loss, octant_mask
from oracle.step import Step, StepParams
from paper_2405_14903_amd.sim import Sim, ellipsoid_poses
from tests.gpu_common import announce, dev, ellipsoid_cfg, host, rel_l2, sphere_cfg

pytestmark = pytest.mark.gpu

# the CG tolerance bench.py runs the rollouts at
BENCH_TOL = 1e-6


@pytest.fixture(scope="module")
def step128():
    announce("oracle: 128^3 moving-ellipsoid step (FP64, solve to 1e-10)")
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=128, steps=1)
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-10, method="mgpcg")
    (c, R), = EllipsoidRollout(prm, sc.u0, sc.theta0, sc.ctrl).poses()
    geo = EllipsoidGeometry(g, c, sc.theta0[3:6], R, sc.ctrl[0, :3], sc.ctrl[0, 3:])
    ref = Step(prm, sc.u0, geo.alpha, geo.us)
    announce(f"  oracle solve: {ref.proj.info[0]} iterations, relative residual {ref.proj.info[1]:.2e}")
    return sc, ref.result


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_step_128_at_bench_tolerance_vs_oracle(step128, precision):
    sc, ref = step128
    announce(f"128^3 step at tol {BENCH_TOL:g}, {precision} V-cycle, against the oracle")
    poses = ellipsoid_poses(sc.theta0, sc.ctrl, sc.dt)
    with Sim(ellipsoid_cfg(sc.n, tol=BENCH_TOL, precision=precision)) as sim:
        u1, st = sim.step(dev(sc.u0), poses[0], sc.ctrl[0])
        torch.cuda.synchronize()
    e = rel_l2(host(u1), ref)
    announce(f"  {st['iters']} CG iterations, true relative residual {st['true_rel_res']:.2e}; "
             f"velocity rel-L2 {e:.2e}")
    assert st["converged"] and e <= 1e-5, (e, st)


@pytest.fixture(scope="module")
def rollout32():
    """The oracle's 64-step rollout of the benchmark scene's 32^3 copy and its gradients."""
    T = 64
    announce(f"oracle: ellipsoid rollout 32^3 x {T} and its adjoint (FP64)")
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=32, steps=T)
    g = Grid(sc.n, sc.dx)
    ro_o = EllipsoidRollout(StepParams(g, sc.dt, tol=1e-11), sc.u0, sc.theta0, sc.ctrl)
    J_o, gT = octant_loss(g, ro_o.forward())
    _, gth_o, gct_o = ro_o.backward(gT)
    return sc, g, J_o, gth_o, gct_o


@pytest.mark.timeout(900)
def test_rollout_gradients_32_at_configuration_length(rollout32):
    """64 steps with a checkpoint every 8 on the 32^3 copy (FP32)."""
    from paper_2405_14903_amd.rollout import EllipsoidRolloutFn
    T, every = 64, 8
    announce(f"ellipsoid rollout gradients 32^3 x {T}, checkpoints every {every}")
    sc, g, J_o, gth_o, gct_o = rollout32
    m = torch.tensor(octant_mask(g), device="cuda")

    with Sim(ellipsoid_cfg(sc.n, tol=1e-7)) as sim:
        u0 = dev(sc.u0)

        def J_gpu(theta0):
            th = torch.tensor(theta0)
            ct = torch.tensor(sc.ctrl)
            uT = EllipsoidRolloutFn.apply(u0, th, ct, sim, every)
            return float((uT.double() ** 2 * m).sum())

        th = torch.tensor(sc.theta0, requires_grad=True)
        ct = torch.tensor(sc.ctrl, requires_grad=True)
        uT = EllipsoidRolloutFn.apply(u0, th, ct, sim, every)
        J = (uT.double() ** 2 * m).sum()
        J.backward()
        torch.cuda.synchronize()
        h = 1e-3
        comps = [0, 4, 7]
        fd = np.array([(J_gpu(sc.theta0 + h * e) - J_gpu(sc.theta0 - h * e)) / (2 * h) for e in np.eye(9)[comps]])
    gth, gct = th.grad.numpy(), ct.grad.numpy()
    e_th, e_ct = rel_l2(gth, gth_o), rel_l2(gct, gct_o)
    e_fd = rel_l2(gth[comps], fd)
    announce(f"  J {float(J):.6f} vs {J_o:.6f}; theta rel {e_th:.2e}, ctrl rel {e_ct:.2e}; "
             f"central differences (h = 1e-3, GPU forward) rel {e_fd:.2e}")
    assert abs(float(J) - J_o) <= 1e-4 * abs(J_o)
    assert e_th <= 1e-3 and e_ct <= 1e-3, (e_th, e_ct)
    # central differences straddle the kinks of the trilinear interpolation and
    # of the marching-squares cases: a few percent, as for the oracle itself
    assert e_fd <= 5e-2, (gth[comps], fd)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_bench_rollout_path_32_against_oracle(rollout32, precision):
    """The rollout exactly as the benchmark drives it (bench tolerance, stored
    pressures replayed, adjoint solves warm-started from the previous adjoint
    pressure) on the 32^3 copy: loss and shape / control gradients against
    the oracle, and against the same rollout with every solve started from
    zero."""
    from paper_2405_14903_amd.rollout import Rollout
    sc, g, J_o, gth_o, gct_o = rollout32
    announce(f"benchmark rollout path 32^3 x 64, {precision}, warm-started adjoint solves, against the oracle")
    out = {}
    with Sim(ellipsoid_cfg(sc.n, tol=BENCH_TOL, precision=precision)) as sim:
        u0 = dev(sc.u0)
        for warm in ("adjoint", False):
            ro = Rollout.ellipsoid(sim, sc.theta0, sc.ctrl, every=8, warm_start=warm)
            J, gT = sim.loss_box(ro.forward(u0))
            ro.backward(gT)
            gth, gct = ro.geometry_gradients()
            out[warm] = (float(J.item()), gth, gct, list(ro.iters["adj"]))
    J, gth, gct, it = out["adjoint"]
    e_th, e_ct = rel_l2(gth, gth_o), rel_l2(gct, gct_o)
    d_th, d_ct = rel_l2(gth, out[False][1]), rel_l2(gct, out[False][2])
    announce(f"  J {J:.6f} vs {J_o:.6f}; theta rel {e_th:.2e}, ctrl rel {e_ct:.2e} against the oracle; "
             f"{d_th:.1e} / {d_ct:.1e} against zero-started solves; adjoint iterations "
             f"{np.mean(it):.2f} warm, {np.mean(out[False][3]):.2f} from zero")
    assert abs(J - J_o) <= 1e-4 * abs(J_o)
    assert e_th <= 1e-3 and e_ct <= 1e-3, (e_th, e_ct)
    assert d_th <= 1e-4 and d_ct <= 1e-4, (d_th, d_ct)


@pytest.fixture(scope="module")
def spheres128():
    announce("oracle: 128^3 twenty-sphere projection (FP64, solve to 1e-10)")
    sc = scenes.scene_spheres_projection(seed=0, n=128, count=20)
    g = Grid(sc.n, sc.dx)
    geo = sphere_geometry(g, sc.spheres)
    k = sc.dt / sc.dx
    pr = Projection(g, sc.u0, geo.alpha, geo.us, k, tol=1e-10, method="mgpcg")
    announce(f"  oracle solve: {pr.info[0]} iterations, relative residual {pr.info[1]:.2e}")
    return sc, g, geo.alpha, pr.ops.G @ pr.P, pr.result


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
def test_precision_configuration_128_vs_oracle_solve(spheres128, precision):
    sc, g, alpha, gp_o, u_o = spheres128
    announce(f"128^3 twenty-sphere projection, {precision} V-cycle, tol {BENCH_TOL:g}, against the oracle solve")
    with Sim(sphere_cfg(sc.n, sc.spheres, tol=BENCH_TOL, precision=precision)) as sim:
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u1, st = sim.project(dev(sc.u0), sc.spheres.ravel(), p_out=P)
        torch.cuda.synchronize()
    gp = Operators(g, alpha).G @ host(P)
    open_ = alpha > 0
    e_gp = rel_l2(gp, gp_o, mask=open_)
    e_u = rel_l2(host(u1), u_o)
    announce(f"  {st['iters']} CG iterations, true relative residual {st['true_rel_res']:.2e}; "
             f"G P rel-L2 {e_gp:.2e}, projected velocity rel-L2 {e_u:.2e}")
    assert st["converged"]
    assert e_u <= 1e-5 and e_gp <= 1e-4, (e_u, e_gp)


def test_octant_loss_and_seed_vs_oracle():
    announce("octant loss and seed against the oracle")
    sc = scenes.scene_sphere_rollout(seed=3, n=32, steps=1)
    g = Grid(sc.n, sc.dx)
    u32 = sc.u0.astype(np.float32)
    J_o, g_o = octant_loss(g, u32.astype(np.float64))
    with Sim(sphere_cfg(sc.n, sc.spheres)) as sim:
        J, gr = sim.loss_box(dev(u32))
        torch.cuda.synchronize()
    announce(f"  J {float(J.item()):.12e} vs {J_o:.12e}")
    # FP64 sums of the same FP32 squares in another order: rounding only
    assert abs(float(J.item()) - J_o) <= 1e-12 * J_o
    # the seed is 2 u on the octant's faces (exact in FP32), 0 elsewhere
    np.testing.assert_array_equal(host(gr), g_o.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("regions", ["auto", "always"])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_closed_box_with_eight_floating_pockets(precision, regions):
    """A sphere of radius 0.74 about the box centre leaves eight corner pockets,
    each a separate closed region with its own constant null vector; the
    projected field and the pressure gradient must match the oracle's, which
    removes the mean per pocket.  "auto": the solver labels the regions after
    the first attempt stalls; "always": labels come with the geometry."""
    announce(f"closed box, eight floating pockets, {precision}, regions {regions}")
    n = 32
    sph = np.array([[0.5, 0.5, 0.5, 0.74]])
    g = Grid((n, n, n), 1.0 / n)
    geo = sphere_geometry(g, sph)
    ops = Operators(g, geo.alpha)
    assert ops.n_floating == 8
    rng = np.random.default_rng(11)
    u = scenes.curl_noise((n, n, n), 1.0 / n, rng) + scenes.face_noise((n, n, n), rng)
    k = 0.5
    pr = Projection(g, u, geo.alpha, geo.us, k, tol=1e-12)
    with Sim(sphere_cfg((n, n, n), sph, tol=1e-7, precision=precision)) as sim:
        sim.set_regions(regions)
        P = torch.empty(g.ncells, dtype=torch.float32, device="cuda")
        u1, st = sim.project(dev(u), sph.ravel(), p_out=P)
        torch.cuda.synchronize()
    e_u = rel_l2(host(u1), pr.result)
    # the pressure gradient enters the velocity as alpha k G P: its error in
    # velocity units, relative to the oracle's velocity (G P itself is two
    # orders smaller than the velocity in these pockets)
    dgp = geo.alpha * k * (ops.G @ (host(P) - pr.P))
    e_gp = float(np.linalg.norm(dgp) / np.linalg.norm(pr.result))
    announce(f"  {st['iters']} CG iterations, true relative residual {st['true_rel_res']:.2e}; "
             f"velocity rel-L2 {e_u:.2e}, alpha k G P error {e_gp:.2e} of |U|")
    assert st["converged"] and e_u <= 1e-5 and e_gp <= 1e-5, (e_u, e_gp, st)


def _same_partition(a, b):
    """Two labellings (-1 = no label) describe the same partition of the cells."""
    a, b = np.asarray(a), np.asarray(b)
    if not np.array_equal(a < 0, b < 0):
        return False
    m = a >= 0
    pairs = np.unique(np.stack([a[m], b[m]]), axis=1)
    return pairs.shape[1] == np.unique(a[m]).size == np.unique(b[m]).size


@pytest.mark.parametrize("case", ["pockets", "pockets_outflow", "spheres_outflow"])
def test_regions_match_oracle_partition(case):
    """Connected fluid regions labelled on the GPU against the oracle's
    (scipy connected components over faces with alpha > 0)."""
    from oracle.mac import WALL, INFLOW, OUTFLOW
    announce(f"connected fluid regions ({case}) against the oracle")
    if case == "pockets":
        n, sph, bc = 32, np.array([[0.5, 0.5, 0.5, 0.74]]), ("wall",) * 6
        obc = (WALL,) * 6
    elif case == "pockets_outflow":
        # the four corner pockets that touch the outflow side are grounded
        n, sph = 32, np.array([[0.5, 0.5, 0.5, 0.74]])
        bc = ("wall", "wall", "wall", "wall", "wall", "outflow")
        obc = (WALL, WALL, WALL, WALL, WALL, OUTFLOW)
    else:
        n = 64
        sph = scenes.random_spheres(np.random.default_rng(7), 32, 0.05, 0.16)
        bc = ("wall", "wall", "wall", "wall", "inflow", "outflow")
        obc = (WALL, WALL, WALL, WALL, INFLOW, OUTFLOW)
    g = Grid((n, n, n), 1.0 / n, bc=obc, inflow_speed=1.0)
    ops = Operators(g, sphere_geometry(g, sph).alpha)
    cfg = sphere_cfg((n, n, n), sph)
    cfg.bc, cfg.inflow_speed = bc, 1.0
    with Sim(cfg) as sim:
        sim.set_geometry(sph.ravel())
        ids, count, floating = sim.regions()
        torch.cuda.synchronize()
        ids = ids.cpu().numpy()
    announce(f"  GPU: {count} regions, {floating} floating; oracle floating {ops.n_floating}")
    assert _same_partition(ids, ops.labels)
    assert floating == ops.n_floating
    # ids are compact and numbered in cell order of each region's first cell
    firsts = [np.flatnonzero(ids == q)[0] for q in range(count)]
    assert count == np.unique(ids[ids >= 0]).size and firsts == sorted(firsts)
