"""Pins for the oracle's MAC grid and gradient matrix."""
import numpy as np

from oracle.mac import Grid, gradient_matrix, WALL, OUTFLOW, PERIODIC, INFLOW


def test_divergence_of_linear_field_is_exact():
    g = Grid((6, 5, 7), 0.2)
    G = gradient_matrix(g)
    x = g.all_face_positions()
    ax = np.concatenate([np.full(g.nf(d), d) for d in range(3)])
    coef = np.array([2.0, -3.0, 5.0])
    u = coef[ax] * x[np.arange(ax.size), ax] + 0.7
    # G^T u = -dx * div u, and div u = 2 - 3 + 5 everywhere
    np.testing.assert_allclose(G.T @ u, -g.dx * coef.sum(), atol=1e-13)


def test_gradient_of_linear_pressure_is_exact():
    g = Grid((5, 6, 4), 0.1, bc=(WALL, WALL, OUTFLOW, WALL, WALL, INFLOW))
    G = gradient_matrix(g)
    xc = g.cell_positions()
    grad = np.array([1.5, -2.0, 0.25])
    p = xc @ grad + 3.0
    gp = G @ p
    side = g.face_side()
    ax = np.concatenate([np.full(g.nf(d), d) for d in range(3)])
    inner = side < 0
    np.testing.assert_allclose(gp[inner], grad[ax[inner]] * g.dx, atol=1e-13)


def test_row_structure_per_boundary_kind():
    g = Grid((4, 3, 5), 0.25, bc=(PERIODIC, PERIODIC, WALL, OUTFLOW, INFLOW, WALL))
    G = gradient_matrix(g)
    nnz = np.diff(G.indptr)
    side = g.face_side()
    assert g.nf(0) == 4 * 3 * 5                   # periodic x: n samples
    assert np.all(nnz[:g.nf(0)] == 2)
    assert np.all(nnz[side >= 0] == 1)
    assert np.all(nnz[side < 0] == 2)
    # every row sums to zero where two cells are present (difference operator)
    rs = np.asarray(G.sum(axis=1)).ravel()
    assert np.all(rs[nnz == 2] == 0)
