"""Independent brute-force forward of the moving-ellipsoid rollout in PyTorch
float64 (dense matrices, dense solve), differentiated by autograd.

It restates the same discrete definitions as the oracle (marching-squares face
fractions, RK2 semi-Lagrangian advection with clamped trilinear interpolation,
cut-cell projection, rigid pose dynamics) in a different form, for tiny closed
boxes only, so that a mistake in the oracle's hand-written adjoint (a dropped
term, a wrong sign, a transposed operand) shows up as a gradient mismatch.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def _skew(v):
    z = torch.zeros((), dtype=v.dtype)
    return torch.stack([torch.stack([z, -v[2], v[1]]), torch.stack([v[2], z, -v[0]]),
                        torch.stack([-v[1], v[0], z])])


def _rot(r):
    t = torch.sqrt(torch.sum(r * r))
    K = _skew(r)
    return torch.eye(3, dtype=F64) + torch.sin(t) / t * K + (1 - torch.cos(t)) / (t * t) * (K @ K)


class TinyBox:
    def __init__(self, n, dx):
        self.n, self.dx = n, dx
        nx, ny, nz = n
        self.shapes = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
        self.nf = [int(np.prod(s)) for s in self.shapes]
        self.F = sum(self.nf)
        self.C = nx * ny * nz
        pos, axis, onwall, corners = [], [], [], []
        G = np.zeros((self.F, self.C))
        f = 0
        for d in range(3):
            sz, sy, sx = self.shapes[d]
            for k in range(sz):
                for j in range(sy):
                    for i in range(sx):
                        ijk = [i, j, k]
                        pos.append([(ijk[a] + (0.0 if a == d else 0.5)) * dx for a in range(3)])
                        axis.append(d)
                        own = ijk[d]
                        onwall.append(own == 0 or own == n[d])
                        if own < n[d]:
                            G[f, i + nx * (j + ny * k)] += 1.0
                        if own >= 1:
                            c = list(ijk)
                            c[d] -= 1
                            G[f, c[0] + nx * (c[1] + ny * c[2])] -= 1.0
                        # cyclic corners (same convention as the face's own plane)
                        t1, t2 = [a for a in range(3) if a != d] if d != 1 else (0, 2)
                        base = list(ijk)
                        cs = []
                        for o1, o2 in ((0, 0), (1, 0), (1, 1), (0, 1)):
                            q = list(base)
                            q[t1] += o1
                            q[t2] += o2
                            cs.append(q[0] + (nx + 1) * (q[1] + (ny + 1) * q[2]))
                        corners.append(cs)
                        f += 1
        self.pos = torch.tensor(pos, dtype=F64)
        self.axis = torch.tensor(axis)
        self.onwall = torch.tensor(onwall)
        self.corners = torch.tensor(corners)
        self.G = torch.tensor(G, dtype=F64)
        kk, jj, ii = np.indices((nz + 1, ny + 1, nx + 1))
        self.nodes = torch.tensor(np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1) * dx, dtype=torch.float64)

    # ---- geometry ----------------------------------------------------------
    def alpha(self, phi_nodes):
        P = phi_nodes[self.corners]                      # (F, 4)
        fl = (P > 0).detach()
        cnt = fl.sum(1)
        out = torch.zeros(self.F, dtype=F64)
        mean = P.mean(1)
        for k in range(4):
            r = [(k + s) % 4 for s in range(4)]
            p0, p1, p2, p3 = P[:, r[0]], P[:, r[1]], P[:, r[2]], P[:, r[3]]
            f0, f1, f2 = fl[:, r[0]], fl[:, r[1]], fl[:, r[2]]

            def safe(a, b):
                dif = (a > 0) != (b > 0)
                den = torch.where(dif, a - b, torch.ones_like(a))
                return torch.where(dif, a / den, torch.zeros_like(a))
            one = (cnt == 1) & f0
            out = out + torch.where(one, 0.5 * safe(p0, p1) * safe(p0, p3), torch.zeros(self.F, dtype=F64))
            three = (cnt == 3) & ~f0
            out = out + torch.where(three, 1 - 0.5 * safe(p0, p1) * safe(p0, p3), torch.zeros(self.F, dtype=F64))
            adj = (cnt == 2) & f0 & f1
            out = out + torch.where(adj, 0.5 * (safe(p0, p3) + safe(p1, p2)), torch.zeros(self.F, dtype=F64))
            if k < 2:
                dg = (cnt == 2) & f0 & f2
                conn = 1 - 0.5 * safe(p1, p0) * safe(p1, p2) - 0.5 * safe(p3, p0) * safe(p3, p2)
                sep = 0.5 * safe(p0, p1) * safe(p0, p3) + 0.5 * safe(p2, p1) * safe(p2, p3)
                out = out + torch.where(dg, torch.where(mean > 0, conn, sep), torch.zeros(self.F, dtype=F64))
        out = torch.where(cnt == 4, torch.ones(self.F, dtype=F64), out)
        return torch.where(self.onwall, torch.zeros(self.F, dtype=F64), out)

    def phi_ellipsoid(self, c, a, R):
        p = (self.nodes - c) @ R
        k0 = torch.sqrt(torch.sum((p / a) ** 2, 1))
        k1 = torch.sqrt(torch.sum((p / a ** 2) ** 2, 1))
        return k0 * (k0 - 1) / k1

    def rigid(self, c, v, w):
        vel = v + torch.cross(w.expand(self.F, 3), self.pos - c, dim=1)
        us = vel.gather(1, self.axis[:, None]).squeeze(1)
        return torch.where(self.onwall, torch.zeros(self.F, dtype=F64), us)

    # ---- advection ---------------------------------------------------------
    def _interp(self, comp, e, x):
        shp = self.shapes[e]
        m = [shp[2], shp[1], shp[0]]
        arr = comp.reshape(shp)
        idx, fr = [], []
        for a in range(3):
            s = x[:, a] / self.dx - (0.0 if a == e else 0.5)
            s = torch.clamp(s, 0.0, m[a] - 1)
            i0 = torch.clamp(torch.floor(s.detach()), max=m[a] - 2).long()
            idx.append(i0)
            fr.append(s - i0)
        out = 0
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    w = ((fr[0] if bx else 1 - fr[0]) * (fr[1] if by else 1 - fr[1])
                         * (fr[2] if bz else 1 - fr[2]))
                    out = out + w * arr[idx[2] + bz, idx[1] + by, idx[0] + bx]
        return out

    def advect(self, u, dt):
        comps = list(torch.split(u, self.nf))
        out = []
        off = 0
        for d in range(3):
            xf = self.pos[off:off + self.nf[d]]
            V = lambda x: torch.stack([self._interp(comps[e], e, x) for e in range(3)], 1)
            xm = xf - 0.5 * dt * V(xf)
            xs = xf - dt * V(xm)
            out.append(self._interp(comps[d], d, xs))
            off += self.nf[d]
        return torch.cat(out)

    # ---- projection --------------------------------------------------------
    def project(self, uhat, alpha, us, k):
        G = self.G
        b = G.T @ (alpha * uhat + (1 - alpha) * us)
        A = G.T @ (alpha[:, None] * G)
        act = (torch.abs(G).T @ alpha > 0).detach()
        ia = torch.nonzero(act).squeeze(1)
        Aa = A[ia][:, ia]
        na = ia.numel()
        # one floating component (closed box): pin its mean to zero
        Aa = Aa + torch.ones(na, na, dtype=F64) / na
        Pa = torch.linalg.solve(Aa, b[ia] / k)
        P = torch.zeros(self.C, dtype=F64).index_put((ia,), Pa)
        return alpha * (uhat - k * (G @ P)) + (1 - alpha) * us


def ellipsoid_rollout_loss(box: TinyBox, u0, theta0, ctrl, dt, octant_lo=0.5):
    c = theta0[0:3]
    a = theta0[3:6]
    R = _rot(theta0[6:9])
    u = u0
    k = dt / box.dx
    for n in range(ctrl.shape[0]):
        v, w = ctrl[n, :3], ctrl[n, 3:]
        c = c + dt * v
        R = _rot(dt * w) @ R
        alpha = box.alpha(box.phi_ellipsoid(c, a, R))
        us = box.rigid(c, v, w)
        u = box.project(box.advect(u, dt), alpha, us, k)
    oct_ = torch.all(box.pos >= octant_lo - 1e-12, dim=1)
    return torch.sum(torch.where(oct_, u * u, torch.zeros_like(u)))
