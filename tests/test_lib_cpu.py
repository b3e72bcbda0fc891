"""Host-side checks of the C-ABI library (no GPU needed): every declared symbol
is exported, descriptor validation, footprints, and the host pose dynamics."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2405_14903_amd import _lib as L
from paper_2405_14903_amd.sim import Config, sim_footprint, ellipsoid_poses, ellipsoid_poses_adjoint
from oracle.rollout import EllipsoidRollout, rodrigues
from oracle.step import StepParams
from oracle.mac import Grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "neuralfluid.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", src, flags=re.M)))


def test_header_and_exports_agree():
    lib = L.load()
    names = _declared()
    assert set(names) == set(L.EXPORTS), names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.sim_version().decode().startswith("neuralfluid")


def _cfg(**kw):
    base = dict(n=(32, 32, 32), dx=1 / 32, dt=1 / 64, geom="spheres", n_spheres=1)
    base.update(kw)
    return Config(**base)


def test_footprint_and_validation():
    f32 = sim_footprint(_cfg())
    f16 = sim_footprint(_cfg(precision="fp16"))
    assert 0 < f16 < 2 * f32 and f32 > 32 ** 3 * 4 * 20
    big = sim_footprint(_cfg(n=(128, 128, 128)))
    assert 50 < big / f32 < 70
    lib = L.load()
    out = C.c_size_t(0)
    for bad, code in [(dict(n=(34, 34, 34)), L.SIM_EINVAL), (dict(dt=0.0), L.SIM_EINVAL),
                      (dict(bc=("periodic",) * 6), L.SIM_EUNSUPPORTED), (dict(n_spheres=0), L.SIM_EINVAL),
                      (dict(tol=-1.0), L.SIM_EINVAL), (dict(max_iter=0), L.SIM_EINVAL)]:
        d = _cfg(**bad).desc()
        assert lib.sim_footprint(C.byref(d), C.byref(out)) == code, bad
    d = _cfg().desc()
    d.nu = 0.1
    assert lib.sim_footprint(C.byref(d), C.byref(out)) == L.SIM_OK      # explicit viscosity
    d.nu = -0.1
    assert lib.sim_footprint(C.byref(d), C.byref(out)) == L.SIM_EINVAL
    assert lib.sim_footprint(None, C.byref(out)) == L.SIM_EINVAL
    # parametric solids: 1 .. SIM_MAX_SOLIDS of them, n_params = 1 + m (1 + 44), no controls
    for m, code in [(0, L.SIM_EINVAL), (1, L.SIM_OK), (L.SIM_MAX_SOLIDS, L.SIM_OK),
                    (L.SIM_MAX_SOLIDS + 1, L.SIM_EINVAL)]:
        d = _cfg(geom="bezier", n_solids=m).desc()
        assert lib.sim_footprint(C.byref(d), C.byref(out)) == code, m
    d = _cfg(geom="bezier", n_solids=2).desc()
    assert d.n_params == 1 + 2 * 45
    d.n_params += 1
    assert lib.sim_footprint(C.byref(d), C.byref(out)) == L.SIM_EINVAL
    d.n_params -= 1
    d.n_ctrl = 6
    assert lib.sim_footprint(C.byref(d), C.byref(out)) == L.SIM_EINVAL
    for n in [(48, 48, 48), (96, 96, 96), (192, 192, 192), (256, 256, 512), (16, 16, 16), (8, 8, 8)]:
        assert sim_footprint(_cfg(n=n)) > 0


def test_pool_arguments_are_checked_before_any_device_call():
    lib = L.load()
    h = C.c_void_p()
    for budget, slots, cells in [(0, 1, 0), (1 << 30, 0, 0), (1 << 30, 65, 0), (1 << 30, 1, -1)]:
        assert lib.sim_pool_create(budget, slots, cells, C.byref(h)) == L.SIM_EINVAL, (budget, slots, cells)
    assert lib.sim_pool_create(1 << 30, 1, 0, None) == L.SIM_EINVAL
    slot, n = C.c_int32(0), C.c_int32(0)
    assert lib.sim_pool_destroy(None) == L.SIM_EINVAL
    assert lib.sim_pool_admit(None, None, None, C.byref(slot)) == L.SIM_EINVAL
    assert lib.sim_pool_tick(None, C.byref(n)) == L.SIM_EINVAL
    assert lib.sim_pool_poll(None, 0, C.byref(n)) == L.SIM_EINVAL
    assert lib.sim_pool_result(None, 0, None, None, None, None, None, None) == L.SIM_EINVAL
    assert lib.sim_status_string(L.SIM_EBUSY).decode().startswith("no free slot")


def test_null_handle_calls_are_rejected():
    lib = L.load()
    assert lib.sim_destroy(None) == L.SIM_EINVAL
    assert lib.sim_step(None, None, None, None, None, None, None, None) == L.SIM_EINVAL
    assert lib.poisson_solve(None, None, None, None, 0.0, 0, None, None) == L.SIM_EINVAL
    assert lib.sim_step_adjoint(None, None, None, None, None, None, None, None, None, None, None) == L.SIM_EINVAL


def test_pose_dynamics_match_oracle():
    rng = np.random.default_rng(0)
    theta0 = np.concatenate([rng.uniform(0.35, 0.65, 3), rng.uniform(0.08, 0.2, 3), rng.standard_normal(3)])
    ctrl = rng.uniform(-0.5, 0.5, (12, 6))
    dt = 1 / 64
    poses = ellipsoid_poses(theta0, ctrl, dt)
    ro = EllipsoidRollout(StepParams(Grid((4, 4, 4), 0.25), dt), None, theta0, ctrl)
    for n, (c, R) in enumerate(ro.poses()):
        np.testing.assert_allclose(poses[n, :3], c, atol=1e-14)
        np.testing.assert_allclose(poses[n, 3:6], theta0[3:6], atol=0)
        np.testing.assert_allclose(poses[n, 6:].reshape(3, 3), R, atol=1e-13)


def test_pose_adjoint_against_central_differences():
    rng = np.random.default_rng(1)
    theta0 = np.concatenate([rng.uniform(0.35, 0.65, 3), rng.uniform(0.08, 0.2, 3), rng.standard_normal(3)])
    T, dt = 7, 0.05
    ctrl = rng.uniform(-0.5, 0.5, (T, 6))
    gs = rng.standard_normal((T, 15))
    gd = rng.standard_normal((T, 6))

    def J(th, ct):
        return float(np.sum(gs * ellipsoid_poses(th, ct, dt)) + np.sum(gd * ct))

    gth, gct = ellipsoid_poses_adjoint(theta0, ctrl, dt, gs, gd)
    h = 1e-6
    for i in range(9):
        e = np.zeros(9)
        e[i] = h
        assert abs((J(theta0 + e, ctrl) - J(theta0 - e, ctrl)) / (2 * h) - gth[i]) < 1e-7 * max(1, abs(gth[i]))
    for (n, j) in [(0, 0), (3, 4), (6, 5), (2, 2)]:
        e = np.zeros_like(ctrl)
        e[n, j] = h
        assert abs((J(theta0, ctrl + e) - J(theta0, ctrl - e)) / (2 * h) - gct[n, j]) < 1e-7 * max(1, abs(gct[n, j]))
