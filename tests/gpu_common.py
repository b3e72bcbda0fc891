"""Shared helpers of the GPU tests: oracle-side scene set-up and comparisons."""
from __future__ import annotations

import sys

import numpy as np
import torch

import scenes
from oracle.mac import Grid
from oracle.geometry import sphere_geometry, EllipsoidGeometry
from oracle.rollout import rodrigues
from paper_2405_14903_amd.sim import Config, Sim


def announce(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a) -> torch.Tensor:
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().double().cpu().numpy()


def rel_l2(a, b, mask=None) -> float:
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    if mask is not None:
        a, b = a[mask], b[mask]
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def sphere_cfg(n, spheres, tol=1e-7, precision="fp32", max_iter=200, dt_factor=0.5):
    n = tuple(n)
    dx = 1.0 / n[0]
    return Config(n=n, dx=dx, dt=dt_factor * dx, geom="spheres", n_spheres=len(spheres), tol=tol,
                  precision=precision, max_iter=max_iter)


def ellipsoid_cfg(n, tol=1e-7, precision="fp32", max_iter=200):
    n = tuple(n)
    dx = 1.0 / n[0]
    return Config(n=n, dx=dx, dt=0.5 * dx, geom="ellipsoid", tol=tol, precision=precision, max_iter=max_iter)


def ellipsoid_step_params(theta_step, ctrl):
    """Oracle geometry for one library step (theta = c, a, R)."""
    c, a, R = theta_step[:3], theta_step[3:6], theta_step[6:].reshape(3, 3)
    return c, a, R, ctrl[:3], ctrl[3:]


def remove_floating_means(ops, p):
    return ops.remove_null(np.where(ops.active, p, 0.0))
