"""Seeded synthetic inputs shared by the GPU library's tests/benchmarks and the oracle.

This module only draws random numbers and arranges them into grid-shaped arrays.
It holds none of the simulation method's arithmetic (no fractions, no
advection, no projection).  Every array is float64 numpy in the canonical
layout used throughout the project:

* velocity: x-faces ``(nz, ny, nx+1)``, then y-faces ``(nz, ny+1, nx)``, then
  z-faces ``(nz+1, ny, nx)``, each raveled with x fastest and concatenated;
* cells: ``(nz, ny, nx)`` raveled with x fastest.

Random-number recipe (numpy ``default_rng(seed)``, PCG64):

* curl noise: a vector potential on MAC edges is drawn i.i.d. N(0,1) in the
  order psi_x, psi_y, psi_z (C order over ``[k][j][i]``), blurred by a
  separable Gaussian (sigma in cells, truncated at 4 sigma, reflecting at the
  domain ends), its tangential components are zeroed on wall planes (so the
  normal velocity on walls is zero), the discrete curl is taken on faces
  (exactly divergence-free), and the field is scaled so max |u_f| = 1;
* scene parameters are drawn after the noise, from the same generator.

Parametric solids (44 values each: origin, rotation matrix, z0, z1, three
key centres, three x eight key radii) are drawn as: origin U[0.35, 0.65]^3,
rotation from a rotation vector uniform in the ball of radius pi (scipy's
Rotation), z0 U[-0.25, -0.12], z1 U[0.12, 0.25], centres U[-0.03, 0.03],
radii U[0.08, 0.16].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.ndimage

__all__ = [
    "face_shapes", "n_faces", "curl_noise", "ellipsoid_theta0", "controls",
    "sphere_center", "random_spheres", "face_noise", "Scene",
    "scene_sphere_rollout", "scene_ellipsoid_rollout", "scene_spheres_projection", "scene_channel",
    "outlet_window_xy", "random_solid", "solids_theta", "scene_solids", "scene_karman",
]


def face_shapes(n):
    nx, ny, nz = n
    return [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]


def n_faces(n):
    return sum(int(np.prod(s)) for s in face_shapes(n))


def _blur(a, sigma):
    if sigma <= 0:
        return a
    return scipy.ndimage.gaussian_filter(a, sigma=sigma, mode="reflect", truncate=4.0)


def curl_noise(n, dx, rng, sigma=2.0, walls=(True, True, True)):
    """Discretely divergence-free random velocity, max |u_f| = 1 (float64, canonical).

    ``walls[a]`` zeroes the potential's tangential components on both domain
    planes normal to axis ``a`` so that the face velocity normal to them is 0.
    """
    nx, ny, nz = n
    psx = _blur(rng.standard_normal((nz + 1, ny + 1, nx)), sigma)
    psy = _blur(rng.standard_normal((nz + 1, ny, nx + 1)), sigma)
    psz = _blur(rng.standard_normal((nz, ny + 1, nx + 1)), sigma)
    if walls[0]:  # planes x = 0, x = X carry psi_y and psi_z
        psy[:, :, 0] = psy[:, :, -1] = 0.0
        psz[:, :, 0] = psz[:, :, -1] = 0.0
    if walls[1]:  # planes y = 0, y = Y carry psi_x and psi_z
        psx[:, 0, :] = psx[:, -1, :] = 0.0
        psz[:, 0, :] = psz[:, -1, :] = 0.0
    if walls[2]:  # planes z = 0, z = Z carry psi_x and psi_y
        psx[0, :, :] = psx[-1, :, :] = 0.0
        psy[0, :, :] = psy[-1, :, :] = 0.0
    ux = (psz[:, 1:, :] - psz[:, :-1, :]) - (psy[1:, :, :] - psy[:-1, :, :])
    uy = (psx[1:, :, :] - psx[:-1, :, :]) - (psz[:, :, 1:] - psz[:, :, :-1])
    uz = (psy[:, :, 1:] - psy[:, :, :-1]) - (psx[:, 1:, :] - psx[:, :-1, :])
    u = np.concatenate([ux.ravel(), uy.ravel(), uz.ravel()]) / dx
    m = np.abs(u).max()
    return u / m if m > 0 else u


def sphere_center(rng, lo=0.35, hi=0.65):
    return rng.uniform(lo, hi, size=3)


def ellipsoid_theta0(rng):
    """(centre c in U[0.35,0.65]^3, semi-axes a in U[0.08,0.2]^3, rotation vector r
    uniform in the ball of radius pi), concatenated as 9 float64."""
    c = rng.uniform(0.35, 0.65, size=3)
    a = rng.uniform(0.08, 0.2, size=3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    r = d * (math.pi * rng.uniform() ** (1.0 / 3.0))
    return np.concatenate([c, a, r])


def controls(rng, steps, lo=-0.5, hi=0.5):
    """Per-step rigid-body controls (v_x, v_y, v_z, w_x, w_y, w_z)."""
    return rng.uniform(lo, hi, size=(steps, 6))


def random_spheres(rng, count=20, rmin=0.03, rmax=0.1):
    """(count, 4) array of (cx, cy, cz, r): centres U[0,1]^3, radii U[rmin, rmax]."""
    c = rng.uniform(0.0, 1.0, size=(count, 3))
    r = rng.uniform(rmin, rmax, size=(count, 1))
    return np.concatenate([c, r], axis=1)


def face_noise(n, rng, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, size=n_faces(n))


def random_solid(rng, lo=0.35, hi=0.65):
    """One parametric solid's 44 parameters (origin, rotation matrix row-major,
    z0, z1, 3 key centres, 3 x 8 key radii)."""
    from scipy.spatial.transform import Rotation
    o = rng.uniform(lo, hi, size=3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    R = Rotation.from_rotvec(d * (math.pi * rng.uniform() ** (1.0 / 3.0))).as_matrix()
    z0, z1 = rng.uniform(-0.25, -0.12), rng.uniform(0.12, 0.25)
    c = rng.uniform(-0.03, 0.03, size=6)
    rho = rng.uniform(0.08, 0.16, size=24)
    return np.concatenate([o, R.ravel(), [z0, z1], c, rho])


def solids_theta(solids, ops=None):
    """Scene vector [m, op_1 .. op_m, solid_1 .. solid_m] (op 0 union, 1 intersection)."""
    m = len(solids)
    ops = [0] * m if ops is None else list(ops)
    return np.concatenate([[float(m)], np.asarray(ops, float), *solids])


@dataclass
class Scene:
    """A seeded scene: grid, time step, solid description and initial velocity."""
    n: tuple
    dx: float
    dt: float
    u0: np.ndarray
    geom: str                       # "none" | "spheres" | "ellipsoid" | "wall" | "bezier"
    spheres: np.ndarray = None      # (m, 4) for geom == "spheres"
    theta0: np.ndarray = None       # (9,) for geom == "ellipsoid"
    ctrl: np.ndarray = None         # (steps, 6) for geom == "ellipsoid"
    steps: int = 1
    extra: dict = field(default_factory=dict)


def scene_sphere_rollout(seed=0, n=32, steps=10):
    """Closed unit box, static sphere r = 0.2 with centre in [0.35,0.65]^3,
    curl-noise initial velocity (sigma = 2 cells), dt = dx/2."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    u0 = curl_noise((n, n, n), dx, rng)
    c = sphere_center(rng)
    sph = np.array([[c[0], c[1], c[2], 0.2]])
    return Scene((n, n, n), dx, 0.5 * dx, u0, "spheres", spheres=sph, steps=steps)


def scene_ellipsoid_rollout(seed=0, n=128, steps=64):
    """Closed unit box with a moving ellipsoid (9 shape parameters, 6 controls per
    step), curl-noise initial velocity, dt = dx/2.  The shape parameters and the
    controls do not depend on ``n`` (same draws at every resolution)."""
    rng = np.random.default_rng(seed)
    theta0 = ellipsoid_theta0(rng)
    ctrl = controls(rng, steps)
    noise_rng = np.random.default_rng([seed, n])
    dx = 1.0 / n
    u0 = curl_noise((n, n, n), dx, noise_rng)
    return Scene((n, n, n), dx, 0.5 * dx, u0, "ellipsoid", theta0=theta0, ctrl=ctrl,
                 steps=steps)


def scene_spheres_projection(seed=0, n=256, count=20):
    """Closed unit box with ``count`` static overlapping spheres.  The field to be
    projected is curl noise plus U[-1,1] noise on every face (adding the noise on
    faces, before the weighted divergence, keeps every connected fluid pocket's
    right-hand side compatible without labelling pockets)."""
    rng = np.random.default_rng(seed)
    sph = random_spheres(rng, count)
    dx = 1.0 / n
    u = curl_noise((n, n, n), dx, rng) + face_noise((n, n, n), rng)
    return Scene((n, n, n), dx, 0.5 * dx, u, "spheres", spheres=sph, steps=1)


# the channel configuration: 1 x 1 x 2 box, 256 x 256 x 512 cells at full size
CHANNEL_LENGTH = (1.0, 1.0, 2.0)
CHANNEL_FULL_N = (256, 256, 512)
CHANNEL_FULL_STEPS = 200


def scene_channel(seed=0, n=(32, 32, 64), steps=200):
    """Inflow / outflow channel with a deformable B-spline wall on the x- side.
    Draws (same at every resolution): 16 x 32 control amplitudes U[0, 1], the
    wall frequency f ~ U[1/T, 2/T] with T = 200 dt of the full-size grid
    (dt = dx/2, dx = 1/256), and the outlet window's phase psi ~ U[0, 2 pi).
    Initial velocity: curl noise with max |u| = 1 (normal component 0 on every
    side).  extra: knots, f, amp (= 0.1), psi."""
    rng = np.random.default_rng(seed)
    knots = rng.uniform(0.0, 1.0, size=(16, 32))
    T = CHANNEL_FULL_STEPS * 0.5 / CHANNEL_FULL_N[0]
    f = rng.uniform(1.0 / T, 2.0 / T)
    psi = rng.uniform(0.0, 2.0 * math.pi)
    n = tuple(int(v) for v in n)
    dx = CHANNEL_LENGTH[0] / n[0]
    noise_rng = np.random.default_rng([seed, *n])
    u0 = curl_noise(n, dx, noise_rng)
    return Scene(n, dx, 0.5 * dx, u0, "wall", steps=steps, extra=dict(knots=knots, f=f, amp=0.1, psi=psi))


def outlet_window_xy(n, dx, psi):
    """Outlet weights (nx * ny, x fastest) of the smooth window over the half
    x > Lx/2: sin^2(2 pi (x/Lx - 1/2)) (1 + sin(2 pi y/Ly + psi) / 2) at the face
    centres, 0 for x <= Lx/2."""
    nx, ny = int(n[0]), int(n[1])
    x = (np.arange(nx) + 0.5) * dx / (nx * dx)
    y = (np.arange(ny) + 0.5) * dx / (ny * dx)
    wx = np.where(x > 0.5, np.sin(2.0 * math.pi * (x - 0.5)) ** 2, 0.0)
    wy = 1.0 + 0.5 * np.sin(2.0 * math.pi * y + psi)
    return (wy[:, None] * wx[None, :]).ravel()


def scene_solids(seed=0, n=32, count=2, ops=None):
    """Closed unit box with a static CSG scene of ``count`` parametric solids
    (``ops`` per solid, default all unions), curl-noise initial velocity,
    dt = dx/2.  The scene vector is ``extra["theta"]``."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    u0 = curl_noise((n, n, n), dx, rng)
    solids = [random_solid(rng) for _ in range(count)]
    return Scene((n, n, n), dx, 0.5 * dx, u0, "bezier", steps=1, extra={"theta": solids_theta(solids, ops)})


KARMAN_BC = ("wall", "wall", "wall", "wall", "inflow", "outflow")


def scene_karman(n=(16, 256, 512), diameter=0.1, speed=1.0, centre=(0.5, 0.4), dt=2e-3, kick=0.1):
    """Flow past a cylinder in a channel, as an x-independent slab: the
    cylinder's axis is the x axis and it spans the slab, the channel is
    [0, 1] across (y, walls) and n_z / n_y along z (inflow at z = 0 with
    ``speed``, outflow at the far end), the slab's x sides are walls.  The
    cylinder is one parametric solid whose eight equal control radii
    D / (2 cos(pi/6)) put its joints on the circle of diameter D (the
    cross-section's radius then stays within 1.4 percent of D / 2).  Initial
    velocity: u_z = speed on every z face, u_x = 0, and a transverse bump
    u_y = kick * speed * exp(-r^2 / D^2) centred 2 D behind the cylinder
    (r the distance in the (y, z) plane; zero on the y walls) that breaks the
    up/down symmetry.  extra: theta, bc, inflow, diameter, centre."""
    n = tuple(int(v) for v in n)
    dx = 1.0 / n[1]
    nx, ny, nz = n
    yc, zc = centre
    # frame: body z -> world x, body x -> world y, body y -> world z
    R = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    rho = diameter / (2.0 * math.cos(math.pi / 6.0))
    solid = np.concatenate([[0.0, yc, zc], R.ravel(), [-1.0, nx * dx + 1.0], np.zeros(6), np.full(24, rho)])
    theta = solids_theta([solid])
    ux = np.zeros((nz, ny, nx + 1))
    k = np.arange(nz)[:, None, None]
    j = np.arange(ny + 1)[None, :, None]
    yy, zz = j * dx, (k + 0.5) * dx
    uy = np.broadcast_to(kick * speed * np.exp(-((yy - yc) ** 2 + (zz - zc - 2 * diameter) ** 2) / diameter ** 2),
                         (nz, ny + 1, nx)).copy()
    uy[:, 0, :] = 0.0
    uy[:, ny, :] = 0.0
    uz = np.full((nz + 1, ny, nx), speed)
    u0 = np.concatenate([ux.ravel(), uy.ravel(), uz.ravel()])
    return Scene(n, dx, dt, u0, "bezier", steps=0,
                 extra=dict(theta=theta, bc=KARMAN_BC, inflow=speed, diameter=diameter, centre=centre))
