"""ctypes loader and signatures for ``libneuralfluid.so`` (see include/neuralfluid.h).

Argument marshalling only.  Loading fails loudly when the library has not been
built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libneuralfluid.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EHIP, SIM_EUNSUPPORTED = 0, -1, -2, -3, -4
SIM_WNOCONV, SIM_WNONFINITE = 1, 2
SIM_SOLVE_HOST, SIM_SOLVE_DEVICE = 0, 1
SIM_REGIONS_AUTO, SIM_REGIONS_ALWAYS, SIM_REGIONS_NEVER = 0, 1, 2
SIM_WARM_PRESSURE, SIM_WARM_ADJOINT = 1, 2
SIM_EBUSY = -5
SIM_EP_FORWARD, SIM_EP_FORWARD_ADJOINT, SIM_EP_PROJECT = 0, 1, 2
SIM_EP_HOST_CHECKED = 1
SIM_FP32, SIM_MIXED_FP16, SIM_MIXED_BF16 = 0, 1, 2
SIM_BC_WALL, SIM_BC_INFLOW, SIM_BC_OUTFLOW, SIM_BC_PERIODIC = 0, 1, 2, 3
SIM_GEOM_NONE, SIM_GEOM_SPHERES, SIM_GEOM_ELLIPSOID, SIM_GEOM_WALL, SIM_GEOM_BEZIER = 0, 1, 2, 3, 4
SIM_MAX_SPHERES = 32
SIM_WALL_KNOTS_Y, SIM_WALL_KNOTS_Z = 16, 32
SIM_MAX_SOLIDS = 8
SIM_BEZIER_SEGMENTS, SIM_BEZIER_SAMPLES, SIM_BEZIER_KEYS, SIM_BEZIER_SHAPE_PARAMS = 4, 16, 3, 44

#: every symbol declared in include/neuralfluid.h
EXPORTS = [
    "sim_version", "sim_status_string", "sim_footprint", "sim_create", "sim_destroy", "sim_layout",
    "sim_step", "sim_step_replay", "sim_project", "sim_step_adjoint", "poisson_solve", "sim_set_geometry",
    "sim_ellipsoid_poses", "sim_ellipsoid_poses_adjoint", "sim_loss_box", "sim_loss_outlet", "sim_profile",
    "sim_profile_read", "sim_set_solve_mode", "sim_set_regions", "sim_regions",
    "sim_loss_box_noalloc", "sim_set_dt", "sim_max_speed", "sim_set_warm_start",
    "sim_pool_create", "sim_pool_destroy", "sim_pool_admit", "sim_pool_tick", "sim_pool_poll", "sim_pool_result",
]

#: sim_kernel ids (include/neuralfluid.h)
KERNELS = ["geom_phi", "geom_alpha", "advect", "rhs", "update", "adj_div", "adj_faces", "advect_adj", "cg_init",
           "cg_apply", "cg_update", "cg_true", "mg_down", "mg_down2", "mg_up1", "mg_up", "mg_coarse", "viscosity"]


class SimDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("dx", C.c_double),
        ("dt", C.c_double),
        ("rho", C.c_double),
        ("nu", C.c_double),
        ("gravity", C.c_double * 3),
        ("bc", C.c_int32 * 6),
        ("inflow_speed", C.c_double),
        ("precision", C.c_int32),
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
        ("geom", C.c_int32),
        ("n_params", C.c_int32),
        ("n_ctrl", C.c_int32),
    ]


class SimStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32),
        ("converged", C.c_int32),
        ("nonfinite", C.c_int32),
        ("pad", C.c_int32),
        ("rel_res", C.c_double),
        ("true_rel_res", C.c_double),
    ]

    def as_dict(self):
        return {"iters": self.iters, "converged": bool(self.converged), "nonfinite": bool(self.nonfinite),
                "rel_res": self.rel_res, "true_rel_res": self.true_rel_res}


class SimEpisode(C.Structure):
    _fields_ = [
        ("desc", SimDesc),
        ("kind", C.c_int32),
        ("steps", C.c_int32),
        ("every", C.c_int32),
        ("flags", C.c_int32),
        ("theta", C.POINTER(C.c_double)),
        ("ctrl", C.POINTER(C.c_double)),
        ("box_lo", C.c_double * 3),
        ("box_hi", C.c_double * 3),
    ]


_lib = None

_vp, _dp, _fp = C.c_void_p, C.POINTER(C.c_double), C.c_void_p


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2405_14903_amd.build` "
                           "(or __graft_entry__.build()) first; there is no fallback implementation")
    lib = C.CDLL(path)
    sig = {
        "sim_version": (C.c_char_p, []),
        "sim_status_string": (C.c_char_p, [C.c_int32]),
        "sim_footprint": (C.c_int32, [C.POINTER(SimDesc), C.POINTER(C.c_size_t)]),
        "sim_create": (C.c_int32, [C.POINTER(SimDesc), C.POINTER(_vp)]),
        "sim_destroy": (C.c_int32, [_vp]),
        "sim_layout": (C.c_int32, [_vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "sim_step": (C.c_int32, [_vp, _fp, _dp, _dp, _fp, _fp, C.POINTER(SimStats), _vp]),
        "sim_project": (C.c_int32, [_vp, _fp, _dp, _dp, _fp, _fp, C.POINTER(SimStats), _vp]),
        "sim_step_replay": (C.c_int32, [_vp, _fp, _dp, _dp, _fp, _fp, _vp]),
        "sim_step_adjoint": (C.c_int32, [_vp, _fp, _fp, _dp, _dp, _fp, _fp, _vp, _vp, C.POINTER(SimStats), _vp]),
        "poisson_solve": (C.c_int32, [_vp, _fp, _fp, _fp, C.c_double, C.c_int32, C.POINTER(SimStats), _vp]),
        "sim_set_geometry": (C.c_int32, [_vp, _dp, _dp, _fp, _vp]),
        "sim_ellipsoid_poses": (C.c_int32, [_dp, _dp, C.c_int32, C.c_double, _dp]),
        "sim_ellipsoid_poses_adjoint": (C.c_int32, [_dp, _dp, C.c_int32, C.c_double, _dp, _dp, _dp, _dp]),
        "sim_loss_box": (C.c_int32, [_vp, _fp, _dp, _dp, _vp, _fp, _vp]),
        "sim_loss_outlet": (C.c_int32, [_vp, _fp, _fp, C.c_double, _vp, _fp, _vp]),
        "sim_profile": (C.c_int32, [_vp, C.c_int32]),
        "sim_profile_read": (C.c_int32, [_vp, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "sim_set_solve_mode": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
        "sim_set_regions": (C.c_int32, [_vp, C.c_int32]),
        "sim_set_dt": (C.c_int32, [_vp, C.c_double]),
        "sim_set_warm_start": (C.c_int32, [_vp, C.c_int32]),
        "sim_pool_create": (C.c_int32, [C.c_size_t, C.c_int32, C.c_int64, C.POINTER(_vp)]),
        "sim_pool_destroy": (C.c_int32, [_vp]),
        "sim_pool_admit": (C.c_int32, [_vp, C.POINTER(SimEpisode), _fp, C.POINTER(C.c_int32)]),
        "sim_pool_tick": (C.c_int32, [_vp, C.POINTER(C.c_int32)]),
        "sim_pool_poll": (C.c_int32, [_vp, C.c_int32, C.POINTER(C.c_int32)]),
        "sim_pool_result": (C.c_int32, [_vp, C.c_int32, _fp, _fp, _vp, _vp, _dp, C.POINTER(SimStats)]),
        "sim_max_speed": (C.c_int32, [_vp, _fp, C.POINTER(C.c_double), _vp]),
        "sim_loss_box_noalloc": (C.c_int32, [C.POINTER(C.c_int32), C.c_double, _fp, _dp, _dp, _vp, _fp, _vp]),
        "sim_regions": (C.c_int32, [_vp, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SolveError(RuntimeError):
    """A call ran to its end but one of its Poisson solves did not reach the
    tolerance or met a NaN / Inf (positive status); ``stats`` holds the
    solver's report when the caller asked for one."""

    def __init__(self, msg, status, stats=None):
        super().__init__(msg)
        self.status, self.stats = status, stats


def check(status: int, what: str, stats=None) -> None:
    if status != SIM_OK:
        msg = load().sim_status_string(status).decode()
        if status > 0:
            raise SolveError(f"{what}: {msg} ({status}); solver report {stats}", status, stats)
        raise RuntimeError(f"{what} failed: {msg} ({status})")
