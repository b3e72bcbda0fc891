"""Why the stored face velocity is the face average (reading of Eq.
u_next_matrix on cut faces), measured on the oracle.

Eq. u_next_matrix calls U^{n+1} = U^ - k G P the fluid velocity, and App. B
Eq. discret_incompress asks the next velocity to be divergence free; on a cut
face (0 < alpha < 1) the two cannot both hold for the fluid velocity W alone,
because the discrete constraint of Eq. projection_matrix balances the fluid
flux alpha W plus the solid flux (1 - alpha) U_s.  The literal reading keeps W
on every face with alpha > 0 (U_s where alpha = 0); this project stores the
face average alpha W + (1 - alpha) U_s, which is exactly divergence free.
The literal reading makes the loss jump whenever a face opens or closes
(W on a nearly closed face is not constrained), so central differences with
h = 1e-3 cross jumps: they disagree with differences too small to cross one,
while the face-average loss gives the same slope at both step sizes.
"""
import numpy as np

import scenes
from oracle.advection import Advection
from oracle.geometry import EllipsoidGeometry
from oracle.mac import Grid
from oracle.projection import Projection
from oracle.rollout import EllipsoidRollout, octant_loss
from oracle.step import StepParams


def _rollout(n, theta0, ctrl, u0, literal):
    g = Grid((n, n, n), 1.0 / n)
    prm = StepParams(g, 0.5 / n, tol=1e-12)
    u = u0
    for k, (c, R) in enumerate(EllipsoidRollout(prm, u0, theta0, ctrl).poses()):
        geo = EllipsoidGeometry(g, c, theta0[3:6], R, ctrl[k, :3], ctrl[k, 3:])
        pr = Projection(g, Advection(g, u, prm.dt).result, geo.alpha, geo.us, prm.k, 1e-12)
        u = np.where(geo.alpha > 0, pr.W, geo.us) if literal else pr.result
        if not literal:
            assert np.linalg.norm(pr.divergence(u)) <= 1e-10 * np.linalg.norm(pr.b)
    return g, u


def test_literal_reading_breaks_central_differences():
    n, T = 16, 3
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=n, steps=T)
    e0 = np.eye(9)[0]                       # the centre's x coordinate
    mismatch = {}
    for literal in (False, True):
        def J(th):
            g, u = _rollout(n, th, sc.ctrl[:T], sc.u0, literal)
            return octant_loss(g, u)[0]
        d3 = (J(sc.theta0 + 1e-3 * e0) - J(sc.theta0 - 1e-3 * e0)) / 2e-3
        d6 = (J(sc.theta0 + 1e-6 * e0) - J(sc.theta0 - 1e-6 * e0)) / 2e-6
        mismatch[literal] = abs(d3 - d6) / abs(d6)
    # measured: 0.24% for the face average, 95% for the literal reading
    assert mismatch[False] < 0.02, mismatch
    assert mismatch[True] > 0.5, mismatch
