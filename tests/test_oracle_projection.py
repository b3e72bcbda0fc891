"""Pins for the oracle's variational pressure projection."""
import numpy as np
import pytest

import scenes
from oracle.mac import Grid, WALL, OUTFLOW, INFLOW, PERIODIC
from oracle.geometry import sphere_geometry, no_solid_geometry, EllipsoidGeometry
from oracle.projection import Projection, Operators, solve
from oracle.rollout import rodrigues
from oracle.step import Step, StepParams

BCS = {
    "closed": (WALL,) * 6,
    "outflow": (WALL, WALL, WALL, WALL, INFLOW, OUTFLOW),
    "periodic": (PERIODIC,) * 6,
}


def _setup(bc, n=6, solid=True, seed=0):
    g = Grid((n, n + 1, n), 1.0 / n, bc=BCS[bc], inflow_speed=0.7)
    rng = np.random.default_rng(seed)
    if solid and bc != "periodic":
        geo = sphere_geometry(g, np.array([[0.45, 0.55, 0.5, 0.27], [0.8, 0.2, 0.3, 0.12]]))
    else:
        geo = no_solid_geometry(g)
        from oracle.geometry import apply_domain_sides
        geo.alpha, geo.us, geo.fixed = apply_domain_sides(g, np.ones(g.nfaces), np.zeros(g.nfaces))
    uhat = rng.uniform(-1, 1, g.nfaces)
    return g, geo, uhat


@pytest.mark.parametrize("bc", ["closed", "outflow", "periodic"])
def test_pcg_matches_dense_direct_solve(bc):
    g, geo, uhat = _setup(bc)
    k = 0.37
    pd = Projection(g, uhat, geo.alpha, geo.us, k, method="dense")
    pc = Projection(g, uhat, geo.alpha, geo.us, k, tol=1e-13)
    assert pd.ops.active.sum() < g.ncells or bc != "closed"
    np.testing.assert_allclose(pc.P, pd.P, atol=1e-10 * np.abs(pd.P).max())
    np.testing.assert_allclose(pc.result, pd.result, atol=1e-11)
    # the dense solution satisfies the system exactly on the active cells
    L = pd.ops.L
    act = pd.ops.active
    b = pd.ops.remove_null(np.where(act, pd.b / k, 0.0))
    np.testing.assert_allclose((L @ pd.P)[act], b[act], atol=1e-11)


@pytest.mark.parametrize("bc", ["closed", "outflow"])
def test_stored_field_divergence_free_and_fluid_velocity_fixed_point(bc):
    g, geo, uhat = _setup(bc, n=8, seed=1)
    pr = Projection(g, uhat, geo.alpha, geo.us, 0.5, tol=1e-13)
    # the balance of Eq. projection_matrix: G^T (S W + (I - S) U_s) = G^T U^{n+1} = 0
    assert np.linalg.norm(pr.divergence(pr.result)) <= 1e-11 * np.linalg.norm(pr.b)
    wd = pr.divergence(geo.alpha * pr.W + (1 - geo.alpha) * geo.us)
    assert np.linalg.norm(wd) <= 1e-11 * np.linalg.norm(pr.b)
    # projecting the fluid velocity again changes nothing
    again = Projection(g, pr.W, geo.alpha, geo.us, 0.5, tol=1e-13)
    assert np.abs(again.P).max() <= 1e-10 * np.abs(pr.P).max()
    np.testing.assert_allclose(again.result, pr.result, atol=1e-11)
    # faces with alpha = 1 follow Eq. u_next_matrix, faces with alpha = 0 the solid
    full, none = geo.alpha == 1.0, geo.alpha == 0.0
    np.testing.assert_allclose(pr.result[full], (uhat - 0.5 * pr.ops.G @ pr.P)[full], atol=1e-14)
    np.testing.assert_array_equal(pr.result[none], geo.us[none])


def test_energy_and_orthogonality_with_static_solid():
    g, geo, uhat = _setup("closed", n=8, seed=2)
    pr = Projection(g, uhat, geo.alpha, geo.us, 1.0, tol=1e-13)
    a = geo.alpha
    e_before = np.sum(a * uhat ** 2)
    e_after = np.sum(a * pr.W ** 2)
    assert e_after <= e_before
    # the fluid velocity is the S-orthogonal projection of U^
    orth = np.sum(a * (uhat - pr.W) * pr.W)
    assert abs(orth) <= 1e-11 * e_before


def test_pressure_constant_shift_leaves_velocity():
    g, geo, uhat = _setup("closed", n=6, seed=3)
    pr = Projection(g, uhat, geo.alpha, geo.us, 0.8, tol=1e-13)
    G = pr.ops.G
    a = geo.alpha
    shifted = np.where(pr.ops.active, pr.P + 3.25, 0.0)
    u2 = a * (uhat - 0.8 * (G @ shifted)) + (1 - a) * geo.us
    np.testing.assert_allclose(u2, pr.result, atol=1e-12)


def test_floating_pocket_components():
    # two disjoint fluid pockets: the projection must handle each null space
    n = 8
    g = Grid((n, n, n), 1.0 / n)
    geo = sphere_geometry(g, np.array([[0.5, 0.5, 0.5, 0.74]]))    # leaves 8 corner pockets
    # add a slab of solid to split the remaining corners: use a second geometry mask
    alpha = geo.alpha.copy()
    ops = Operators(g, alpha)
    rng = np.random.default_rng(4)
    uhat = rng.uniform(-1, 1, g.nfaces)
    pr = Projection(g, uhat, alpha, geo.us, 1.0, tol=1e-13)
    assert ops.n_floating == 8
    assert np.linalg.norm(pr.divergence(pr.result)) <= 1e-10 * np.linalg.norm(pr.b)
    pd = Projection(g, uhat, alpha, geo.us, 1.0, method="dense")
    np.testing.assert_allclose(pr.result, pd.result, atol=1e-10)


def test_rest_stays_at_rest():
    n = 10
    g = Grid((n, n, n), 1.0 / n)
    geo = sphere_geometry(g, np.array([[0.5, 0.45, 0.55, 0.2]]))
    st = Step(StepParams(g, 0.05), np.zeros(g.nfaces), geo.alpha, geo.us)
    assert np.all(st.result == 0.0)


def test_hydrostatic_balance():
    n = 8
    g = Grid((n, n, n), 1.0 / n)
    geo = sphere_geometry(g, np.array([[0.5, 0.5, 0.5, 0.22]]))
    prm = StepParams(g, 0.05, gravity=(0.0, 0.0, -9.8), tol=1e-13)
    st = Step(prm, np.zeros(g.nfaces), geo.alpha, geo.us)
    assert np.abs(st.result).max() <= 1e-11
    # the pressure is the discrete linear potential: k (G P) = dt g on faces carrying fluid
    gp = prm.k * (st.proj.ops.G @ st.P)
    zf = np.concatenate([np.zeros(g.nf(0) + g.nf(1)), np.ones(g.nf(2))])
    m = geo.alpha > 0
    np.testing.assert_allclose(gp[m], (-9.8 * 0.05 * zf)[m], atol=1e-11)


@pytest.mark.parametrize("bc", ["closed", "outflow", "periodic"])
def test_mgpcg_matches_dense_direct_solve(bc):
    # a deep hierarchy (coarsest level of at most 8 unknowns) on a tiny grid:
    # the multigrid only preconditions CG, the answer is the dense solution
    from oracle.projection import mgpcg, dense_solve
    g, geo, uhat = _setup(bc, seed=5)
    ops = Operators(g, geo.alpha)
    b = ops.remove_null(np.where(ops.active, ops.GT @ (geo.alpha * uhat + (1 - geo.alpha) * geo.us), 0.0))
    xd = ops.remove_null(dense_solve(ops.L, b, ops.active))
    xm, it, rel = mgpcg(ops.L, b, ops.active, g.n, 1e-13, coarsest=8)
    xm = ops.remove_null(xm)
    assert rel <= 1e-13 and it > 0
    np.testing.assert_allclose(xm, xd, atol=1e-10 * np.abs(xd).max())


def test_mgpcg_matches_pcg_with_pockets_and_outflow():
    from oracle.projection import mgpcg, pcg
    n = 16
    rng = np.random.default_rng(6)
    for bc in [(WALL,) * 6, (WALL, WALL, WALL, WALL, INFLOW, OUTFLOW)]:
        g = Grid((n, n, n), 1.0 / n, bc=bc, inflow_speed=0.5)
        geo = sphere_geometry(g, np.array([[0.5, 0.5, 0.5, 0.74]]))
        ops = Operators(g, geo.alpha)
        if bc[5] == WALL:
            assert ops.n_floating == 8
        b = ops.remove_null(np.where(ops.active, rng.uniform(-1, 1, g.ncells), 0.0))
        xp, _, _ = pcg(ops.L, b, ops.active, 1e-13)
        xm, it, rel = mgpcg(ops.L, b, ops.active, g.n, 1e-13, coarsest=16)
        assert rel <= 1e-13
        xp, xm = ops.remove_null(xp), ops.remove_null(xm)
        np.testing.assert_allclose(xm, xp, atol=1e-9 * np.abs(xp).max())
