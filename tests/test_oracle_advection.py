"""Pins for the oracle's semi-Lagrangian advection."""
import math

import numpy as np

import scenes
from oracle.mac import Grid
from oracle.advection import Advection


def _assemble(g, comp):
    return np.concatenate([c.ravel() for c in comp])


def test_constant_field_stays_constant():
    g = Grid((6, 5, 7), 1.0 / 7)
    u = np.concatenate([np.full(g.nf(0), 0.3), np.full(g.nf(1), -0.8), np.full(g.nf(2), 0.45)])
    out = Advection(g, u, 0.05).result
    np.testing.assert_allclose(out, u, atol=1e-15)


def test_linear_field_translated_by_uniform_flow():
    # u = (U0, c x, 0): exact solution u_y(x, t + dt) = c (x - U0 dt)
    n = 12
    g = Grid((n, n, n), 1.0 / n)
    U0, c, dt = 0.6, 0.9, 0.5 / n
    xs = [g.face_positions(d) for d in range(3)]
    u = np.concatenate([np.full(g.nf(0), U0), c * xs[1][:, 0], np.zeros(g.nf(2))])
    out = g.split(Advection(g, u, dt).result)
    exact_y = c * (xs[1][:, 0] - U0 * dt)
    # away from the upstream x boundary (where the trace leaves the lattice)
    keep = xs[1][:, 0] - 2 * U0 * dt > 0.5 * g.dx
    np.testing.assert_allclose(out[1].ravel()[keep], exact_y[keep], atol=1e-14)
    np.testing.assert_allclose(out[0].ravel(), U0, atol=1e-15)


def test_integer_cell_shift_is_exact():
    # uniform flow of one cell per step along x carries every component one cell
    n = 8
    g = Grid((n, n, n), 1.0 / n)
    dt = 0.5 / n
    U0 = g.dx / dt
    rng = np.random.default_rng(0)
    u = np.concatenate([np.full(g.nf(0), U0), np.zeros(g.nf(1)), np.zeros(g.nf(2))])
    # passive check through the interpolation itself: with v = (U0, 0, 0) the source
    # point of every face is exactly one cell upstream
    from oracle.advection import Interp
    xf = g.face_positions(1)
    comp = rng.standard_normal(g.nf(1))
    vals = Interp(g, 1, xf - np.array([g.dx, 0.0, 0.0])).value(comp)
    sh = comp.reshape(g.face_shape(1))
    expect = np.concatenate([sh[:, :, :1], sh[:, :, :-1]], axis=2).ravel()   # clamped at i = 0
    np.testing.assert_allclose(vals, expect, atol=1e-15)
    out = Advection(g, u, dt).result
    np.testing.assert_allclose(out, u, atol=1e-14)


def _trilinear_scalar(arr, s):
    """Pure-Python trilinear sample of arr[k][j][i] at index coords s=(si,sj,sk),
    clamped to the lattice (independent re-statement)."""
    m = (arr.shape[2], arr.shape[1], arr.shape[0])
    idx, fr = [], []
    for a in range(3):
        v = min(max(s[a], 0.0), m[a] - 1)
        i0 = min(int(math.floor(v)), m[a] - 2)
        idx.append(i0)
        fr.append(v - i0)
    tot = 0.0
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                w = ((fr[0] if bx else 1 - fr[0]) * (fr[1] if by else 1 - fr[1])
                     * (fr[2] if bz else 1 - fr[2]))
                tot += w * arr[idx[2] + bz, idx[1] + by, idx[0] + bx]
    return tot


def test_brute_force_rk2_at_tiny_size():
    n = (4, 3, 5)
    g = Grid(n, 0.25)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, g.nfaces)
    dt = 0.2
    comps = g.split(u)
    offs = [[0.0 if a == e else 0.5 for a in range(3)] for e in range(3)]

    def V(x):
        return [_trilinear_scalar(comps[e], [x[a] / g.dx - offs[e][a] for a in range(3)])
                for e in range(3)]

    expect = []
    for d in range(3):
        for xf in g.face_positions(d):
            v0 = V(xf)
            xm = [xf[a] - 0.5 * dt * v0[a] for a in range(3)]
            v1 = V(xm)
            xs = [xf[a] - dt * v1[a] for a in range(3)]
            expect.append(_trilinear_scalar(comps[d], [xs[a] / g.dx - offs[d][a] for a in range(3)]))
    np.testing.assert_allclose(Advection(g, u, dt).result, expect, atol=1e-14)


def test_tangent_fd_and_adjoint_identity():
    n = 10
    g = Grid((n, n, n), 1.0 / n)
    rng = np.random.default_rng(6)
    u = scenes.curl_noise(g.n, g.dx, rng)
    dt = 0.5 / n
    adv = Advection(g, u, dt)
    v = rng.standard_normal(g.nfaces)
    w = rng.standard_normal(g.nfaces)
    jv = adv.jvp(v)
    h = 1e-7
    fd = (Advection(g, u + h * v, dt).result - Advection(g, u - h * v, dt).result) / (2 * h)
    # faces on the walls trace back along the wall plane itself, where the clamp
    # has a kink (one-sided derivatives differ); the projection overwrites them
    inner = g.face_side() < 0
    assert inner.sum() == g.nfaces - 6 * n * n
    np.testing.assert_allclose(jv[inner], fd[inner], atol=2e-6)
    lhs, rhs = jv @ w, v @ adv.vjp(w)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
