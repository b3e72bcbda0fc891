"""Variational pressure projection with cut-cell face fractions (FP64 oracle;
test infrastructure only).

Paper, Sec. Projection: with S = diag(alpha) and k = dt / (rho dx),

    (Eq. projection_matrix)  k G^T S G P = G^T S U^ + G^T (I - S) U_s
    (Eq. u_next_matrix)      U^{n+1}     = U^ - k G P

i.e. the fluid flux alpha u plus the solid flux (1 - alpha) u_s through the
faces of every cell balances.  Readings (listed in the design notes):

* the fluid velocity of a face is W = U^ - k G P (Eq. u_next_matrix); the
  velocity stored on a face is its area average over the fluid and solid
  parts, U^{n+1} = alpha W + (1 - alpha) U_s.  On fully fluid faces this is
  Eq. u_next_matrix itself; on faces with alpha = 0 it is the solid velocity;
  it is continuous in alpha (so in the shape parameters), and the stored
  field is exactly divergence free, G^T U^{n+1} = 0 -- which is the balance
  of Eq. projection_matrix;
* cells with sum(alpha over their faces) = 0 are inactive (fully solid) and
  carry no pressure unknown;
* a connected set of active cells (joined through faces with alpha > 0) that
  touches no Dirichlet (OUTFLOW) face has a constant null vector; its pressure
  is taken with zero mean, and its right-hand side must sum to zero there
  (compatible) -- the solve removes the rounding-level mean first;
* the solve is any converged FP64 solver: the result is the solution of the
  linear system.  Here: Jacobi-preconditioned CG written out plainly, stopped on
  the true relative residual ||b - A x|| / ||b||; the same CG preconditioned
  by an aggregation multigrid V-cycle for large grids (a faster route to the
  same solution: only the preconditioner differs); a dense least-squares
  solve serves for tiny grids.

Pinned by: tests/test_oracle_projection.py (dense direct solve at tiny sizes
with solids, walls, outflow and periodic sides; zero divergence of the stored
field; the fluid velocity is a fixed point of a second projection; energy
decrease and S-orthogonality of the fluid velocity; constant shifts of P leave
U unchanged; rest and hydrostatic cases).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

from .mac import Grid, gradient_matrix


class Operators:
    """G, S-weighted operator pieces and the connectivity of active cells."""

    def __init__(self, grid: Grid, alpha: np.ndarray):
        self.grid = grid
        self.alpha = alpha
        self.G = gradient_matrix(grid)
        self.GT = self.G.T.tocsr()
        S = sp.diags(alpha)
        self.L = (self.GT @ S @ self.G).tocsr()          # G^T S G (unit scale)
        absG = abs(self.G)
        self.diag = absG.T @ alpha                       # sum of alpha over a cell's faces
        self.active = self.diag > 0.0
        self.mask = alpha > 0.0                          # faces carrying fluid
        # connectivity through faces with alpha > 0 joining two cells
        two = np.asarray(absG.sum(axis=1)).ravel() == 2
        link = (two & self.mask)
        Gl = self.G[link]
        coo = Gl.tocoo()
        rows = coo.row.reshape(-1) if coo.nnz else np.zeros(0, int)
        cols = coo.col
        # each linking face has exactly two entries: pair them
        order = np.argsort(rows, kind="stable")
        cols = cols[order]
        a_ = cols[0::2]
        b_ = cols[1::2]
        n = grid.ncells
        adj = sp.coo_matrix((np.ones(a_.size), (a_, b_)), shape=(n, n))
        ncomp, labels = csgraph.connected_components(adj, directed=False)
        self.labels = np.where(self.active, labels, -1)
        # grounded: the component has a face with alpha > 0 and a single cell (Dirichlet ghost)
        one = np.asarray(absG.sum(axis=1)).ravel() == 1
        dir_faces = one & self.mask
        grounded_cells = np.unique(absG[dir_faces].tocoo().col)
        grounded = np.zeros(ncomp, bool)
        grounded[labels[grounded_cells]] = True
        floating = self.active & ~grounded[labels]
        _, compact = np.unique(labels[floating], return_inverse=True)
        self.float_label = np.full(n, -1, np.int64)
        self.float_label[floating] = compact
        self.n_floating = int(compact.max()) + 1 if compact.size else 0

    def remove_null(self, v):
        """Remove the mean over every floating component (returns a copy)."""
        v = np.array(v, dtype=np.float64, copy=True)
        sel = self.float_label >= 0
        if self.n_floating:
            lab = self.float_label[sel]
            sums = np.bincount(lab, weights=v[sel], minlength=self.n_floating)
            cnt = np.bincount(lab, minlength=self.n_floating)
            v[sel] -= (sums / cnt)[lab]
        return v

    def apply(self, x):
        return self.L @ x


def pcg(L, b, active, tol, max_iter=100000):
    """Jacobi-preconditioned CG on the active cells; stops on the true relative
    residual.  Returns (x, iterations, relative residual)."""
    idx = np.flatnonzero(active)
    A = L[idx][:, idx].tocsr()
    bb = b[idx]
    nb = np.linalg.norm(bb)
    x = np.zeros(b.size)
    if nb == 0.0:
        return x, 0, 0.0
    dinv = 1.0 / A.diagonal()
    xa = np.zeros(idx.size)
    r = bb.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    rel = 1.0
    while it < max_iter:
        q = A @ p
        a = rz / (p @ q)
        xa += a * p
        r -= a * q
        it += 1
        if np.linalg.norm(r) <= tol * nb:
            rt = bb - A @ xa                      # confirm on the true residual
            rel = np.linalg.norm(rt) / nb
            if rel <= tol:
                break
            r = rt
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    x[idx] = xa
    return x, it, rel


def aggregation_hierarchy(n, active, A, coarsest=512):
    """Operators of an aggregation multigrid on the active cells: level l+1
    has one unknown per 2x2x2 block of level l (blocks without an active cell
    dropped), P_l is the piecewise-constant prolongation and A_{l+1} =
    P_l^T A_l P_l (Galerkin).  Returns ([A_0, A_1, ...], [P_0, ...])."""
    idx = np.flatnonzero(active)
    nx, ny, nz = n
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    ops, proj = [A], []
    while ops[-1].shape[0] > coarsest:
        i, j, k = i // 2, j // 2, k // 2
        key = i + (nx // 2 + 1) * (j + (ny // 2 + 1) * k)
        nx, ny, nz = nx // 2 + 1, ny // 2 + 1, nz // 2 + 1
        uniq, agg = np.unique(key, return_inverse=True)
        if uniq.size >= ops[-1].shape[0]:
            break
        P = sp.csr_matrix((np.ones(agg.size), (np.arange(agg.size), agg)), shape=(agg.size, uniq.size))
        proj.append(P)
        ops.append((P.T @ ops[-1] @ P).tocsr())
        kk = uniq
        i, j, k = kk % nx, (kk // nx) % ny, kk // (nx * ny)
    return ops, proj


def vcycle(ops, proj, dinv, coarse_pinv, r, level=0, omega=2.0 / 3.0, sweeps=2):
    """One V-cycle for A_level z = r from z = 0: damped-Jacobi sweeps before
    and after the coarse-grid correction (the same sweeps both ways, so the
    cycle is a symmetric operator), exact (pseudo-inverse) coarsest solve."""
    if level == len(proj):
        return coarse_pinv @ r
    A, D = ops[level], dinv[level]
    z = omega * D * r
    for _ in range(sweeps - 1):
        z = z + omega * D * (r - A @ z)
    P = proj[level]
    z = z + P @ vcycle(ops, proj, dinv, coarse_pinv, P.T @ (r - A @ z), level + 1, omega, sweeps)
    for _ in range(sweeps):
        z = z + omega * D * (r - A @ z)
    return z


def mgpcg(L, b, active, n, tol, max_iter=10000, coarsest=512):
    """CG preconditioned by the aggregation V-cycle on the active cells; stops
    on the true relative residual.  Returns (x, iterations, relative residual)."""
    idx = np.flatnonzero(active)
    A = L[idx][:, idx].tocsr()
    bb = b[idx]
    nb = np.linalg.norm(bb)
    x = np.zeros(b.size)
    if nb == 0.0:
        return x, 0, 0.0
    ops, proj = aggregation_hierarchy(n, active, A, coarsest)
    # an aggregate that covers a whole floating pocket has a zero row (the
    # pocket's constant is in the null space): it gets no smoothing
    dinv = []
    for M in ops:
        dg = M.diagonal()
        keep = dg > 1e-12 * A.diagonal().max()
        dinv.append(np.where(keep, 1.0 / np.where(keep, dg, 1.0), 0.0))
    # pseudo-inverse of the coarsest operator; eigenvalues at rounding level
    # of the finest operator's scale (constants of floating pockets) count as 0
    w, V = np.linalg.eigh(ops[-1].toarray())
    cut = 1e-12 * A.diagonal().max()
    winv = np.where(np.abs(w) > cut, 1.0 / np.where(np.abs(w) > cut, w, 1.0), 0.0)
    coarse_pinv = (V * winv) @ V.T
    xa = np.zeros(idx.size)
    r = bb.copy()
    z = vcycle(ops, proj, dinv, coarse_pinv, r)
    p = z.copy()
    rz = r @ z
    it, rel = 0, 1.0
    while it < max_iter:
        q = A @ p
        a = rz / (p @ q)
        xa += a * p
        r -= a * q
        it += 1
        if np.linalg.norm(r) <= tol * nb:
            rt = bb - A @ xa
            rel = np.linalg.norm(rt) / nb
            if rel <= tol:
                break
            r = rt
        z = vcycle(ops, proj, dinv, coarse_pinv, r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    x[idx] = xa
    return x, it, rel


def dense_solve(L, b, active):
    """Minimum-norm least-squares solve on the active cells (tiny grids only)."""
    idx = np.flatnonzero(active)
    A = L[idx][:, idx].toarray()
    x = np.zeros(b.size)
    x[idx] = np.linalg.lstsq(A, b[idx], rcond=None)[0]
    return x


def solve(ops: Operators, b, tol=1e-12, method="pcg"):
    """Solve (G^T S G) x = b with zero mean on floating components."""
    b = ops.remove_null(np.where(ops.active, b, 0.0))
    if method == "dense":
        x = dense_solve(ops.L, b, ops.active)
        info = (0, 0.0)
    elif method == "mgpcg":
        x, it, rel = mgpcg(ops.L, b, ops.active, ops.grid.n, tol)
        info = (it, rel)
    else:
        x, it, rel = pcg(ops.L, b, ops.active, tol)
        info = (it, rel)
    return ops.remove_null(x), info


class Projection:
    """Eq. projection_matrix + Eq. u_next_matrix, with tangent and adjoint.

    ``uhat``: advected (+ viscous) face velocity; ``us``: solid face velocity;
    ``alpha``: face fractions.  ``k = dt / (rho dx)``.  ``W`` is the fluid
    velocity, ``result`` the stored face-average velocity.
    """

    def __init__(self, grid: Grid, uhat, alpha, us, k, tol=1e-12, method="pcg"):
        self.grid, self.k, self.tol, self.method = grid, k, tol, method
        self.uhat, self.alpha, self.us = uhat, alpha, us
        self.ops = ops = Operators(grid, alpha)
        # right-hand side of Eq. projection_matrix (divided by k: unit-scaled system)
        self.b = ops.GT @ (alpha * uhat + (1.0 - alpha) * us)
        self.P, self.info = solve(ops, self.b / k, tol, method)
        self.W = uhat - k * (ops.G @ self.P)
        self.result = alpha * self.W + (1.0 - alpha) * us

    def divergence(self, u):
        """G^T u (= -dx * discrete divergence): zero for the stored field."""
        return self.ops.GT @ u

    def jvp(self, duhat, dalpha, dus):
        ops, k, a = self.ops, self.k, self.alpha
        # d b = G^T (S duhat + (I-S) dus + dS (uhat - us));  d(L) P = G^T dS G P
        GP = ops.G @ self.P
        db = ops.GT @ (a * duhat + (1.0 - a) * dus + dalpha * (self.uhat - self.us))
        rhs = db / k - ops.GT @ (dalpha * GP)
        dP, _ = solve(ops, rhs, self.tol, self.method)
        dW = duhat - k * (ops.G @ dP)
        return a * dW + dalpha * (self.W - self.us) + (1.0 - a) * dus

    def vjp(self, g):
        """Returns (dJ/duhat, dJ/dalpha, dJ/dus) for dJ/dU^{n+1} = g.

        Derived as the transpose of the forward map (Sec. Back-propagation
        through Time, Projection paragraph, and through Geometry), with
        A = k G^T S G:
          dJ/dP = -k G^T S g;  A y = dJ/dP;  h = g + G y;
          dJ/dU^ = S h;  dJ/dU_s = (I - S) h;  dJ/dalpha_f = h_f (W_f - U_s,f).
        """
        ops, k, a = self.ops, self.k, self.alpha
        gP = -k * (ops.GT @ (a * g))
        y, _ = solve(ops, gP / k, self.tol, self.method)    # A y = gP  <=>  (G^T S G) y = gP / k
        h = g + ops.G @ y
        self.y = y
        return a * h, h * (self.W - self.us), (1.0 - a) * h
