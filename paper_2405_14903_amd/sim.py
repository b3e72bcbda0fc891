"""PyTorch-facing binding of the C ABI: argument checking and marshalling.

Every array is a CUDA/HIP torch tensor handed to the library by pointer on the
caller's current stream; shapes, dtypes and devices are checked here before
any pointer crosses the ABI (a wrong size would otherwise be an out-of-bounds
access on the GPU).  No numerical work happens in Python.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from ._lib import SolveError  # noqa: F401  (re-exported)

_BC = {"wall": L.SIM_BC_WALL, "inflow": L.SIM_BC_INFLOW, "outflow": L.SIM_BC_OUTFLOW,
       "periodic": L.SIM_BC_PERIODIC}
_PREC = {"fp32": L.SIM_FP32, "fp16": L.SIM_MIXED_FP16, "bf16": L.SIM_MIXED_BF16}
_GEOM = {"none": L.SIM_GEOM_NONE, "spheres": L.SIM_GEOM_SPHERES, "ellipsoid": L.SIM_GEOM_ELLIPSOID,
         "wall": L.SIM_GEOM_WALL, "bezier": L.SIM_GEOM_BEZIER}


@dataclass
class Config:
    n: tuple
    dx: float
    dt: float
    rho: float = 1.0
    nu: float = 0.0
    gravity: tuple = (0.0, 0.0, 0.0)
    bc: tuple = ("wall",) * 6
    inflow_speed: float = 0.0
    precision: str = "fp32"
    tol: float = 1e-6
    max_iter: int = 200
    geom: str = "none"
    n_spheres: int = 0
    n_solids: int = 0           # "bezier": parametric solids in the CSG scene

    def desc(self) -> L.SimDesc:
        d = L.SimDesc()
        for a in range(3):
            d.n[a] = int(self.n[a])
            d.gravity[a] = float(self.gravity[a])
        d.dx, d.dt, d.rho, d.nu = float(self.dx), float(self.dt), float(self.rho), float(self.nu)
        for s in range(6):
            b = self.bc[s]
            d.bc[s] = _BC[b] if isinstance(b, str) else int(b)
        d.inflow_speed = float(self.inflow_speed)
        d.precision = _PREC[self.precision] if isinstance(self.precision, str) else int(self.precision)
        d.tol, d.max_iter = float(self.tol), int(self.max_iter)
        d.geom = _GEOM[self.geom] if isinstance(self.geom, str) else int(self.geom)
        if d.geom == L.SIM_GEOM_SPHERES:
            d.n_params, d.n_ctrl = 4 * int(self.n_spheres), 0
        elif d.geom == L.SIM_GEOM_ELLIPSOID:
            d.n_params, d.n_ctrl = 15, 6
        elif d.geom == L.SIM_GEOM_WALL:
            d.n_params, d.n_ctrl = L.SIM_WALL_KNOTS_Y * L.SIM_WALL_KNOTS_Z, 3
        elif d.geom == L.SIM_GEOM_BEZIER:
            d.n_params, d.n_ctrl = 1 + int(self.n_solids) * (1 + L.SIM_BEZIER_SHAPE_PARAMS), 0
        else:
            d.n_params, d.n_ctrl = 0, 0
        return d

    @property
    def nfaces(self):
        nx, ny, nz = self.n
        return (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)

    @property
    def ncells(self):
        nx, ny, nz = self.n
        return nx * ny * nz


def _ptr(t: torch.Tensor | None, n: int, dtype, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected contiguous {dtype} with {n} elements, got {t.dtype} "
                         f"{tuple(t.shape)} contiguous={t.is_contiguous()}")
    return C.c_void_p(t.data_ptr())


def _host_doubles(a, n: int, name: str):
    if n == 0:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
    if arr.size != n:
        raise ValueError(f"{name}: expected {n} values, got {arr.size}")
    return arr, arr.ctypes.data_as(C.POINTER(C.c_double))


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceStats:
    """Solver report that a kernel writes into pinned host memory (device
    solve mode); valid once the stream the call was enqueued on has reached
    it.  ``as_dict()`` synchronises that stream first."""

    def __init__(self):
        self.buf = torch.zeros(C.sizeof(L.SimStats), dtype=torch.uint8, pin_memory=True)
        self.stream = torch.cuda.current_stream()

    def ptr(self):
        return C.cast(C.c_void_p(self.buf.data_ptr()), C.POINTER(L.SimStats))

    def as_dict(self):
        self.stream.synchronize()
        return L.SimStats.from_buffer_copy(bytes(self.buf.numpy().tobytes())).as_dict()


def sim_footprint(cfg: Config) -> int:
    lib = L.load()
    out = C.c_size_t(0)
    d = cfg.desc()
    L.check(lib.sim_footprint(C.byref(d), C.byref(out)), "sim_footprint")
    return int(out.value)


class Sim:
    """One library handle (workspace for one grid / configuration)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        self.lib = L.load()
        self._desc = cfg.desc()
        h = C.c_void_p()
        L.check(self.lib.sim_create(C.byref(self._desc), C.byref(h)), "sim_create")
        self.h = h
        self.nf, self.nc = cfg.nfaces, cfg.ncells
        self.n_params, self.n_ctrl = self._desc.n_params, self._desc.n_ctrl
        self.dt = float(cfg.dt)

    def close(self):
        if self.h is not None and self.h.value:
            self.lib.sim_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- entry points --------------------------------------------------
    def set_dt(self, dt: float):
        """Time step of the handle's later calls (CFL sub-stepping)."""
        L.check(self.lib.sim_set_dt(self.h, float(dt)), "sim_set_dt")
        self.dt = float(dt)

    def max_speed(self, u) -> float:
        """Largest |u_f| over the faces (waits on the stream)."""
        v = C.c_double(0.0)
        L.check(self.lib.sim_max_speed(self.h, _ptr(u, self.nf, torch.float32, "u"), C.byref(v), _stream()),
                "sim_max_speed")
        return v.value

    def set_warm_start(self, pressure: bool = False, adjoint: bool = False):
        """Start each pressure solve from the previous step's pressure and / or
        each adjoint solve from the previous adjoint pressure (same tolerance;
        the held pressures are forgotten by every call, so the next solves
        start from zero)."""
        kinds = (L.SIM_WARM_PRESSURE if pressure else 0) | (L.SIM_WARM_ADJOINT if adjoint else 0)
        L.check(self.lib.sim_set_warm_start(self.h, kinds), "sim_set_warm_start")

    def set_solve_mode(self, mode: str = "host", budget: int = 0):
        """"host": solves wait on the stream for convergence checks (default);
        "device": nothing waits on the host, each solve runs at most
        min(max_iter, budget) iterations and its report is written on the
        device (stats come back as :class:`DeviceStats`)."""
        m = {"host": L.SIM_SOLVE_HOST, "device": L.SIM_SOLVE_DEVICE}[mode]
        L.check(self.lib.sim_set_solve_mode(self.h, m, int(budget)), "sim_set_solve_mode")
        self.device_mode = m == L.SIM_SOLVE_DEVICE

    def set_regions(self, mode: str = "auto"):
        """Connected-region labelling: "auto" (label after a stalled solve),
        "always" (at every geometry evaluation) or "never"."""
        m = {"auto": L.SIM_REGIONS_AUTO, "always": L.SIM_REGIONS_ALWAYS, "never": L.SIM_REGIONS_NEVER}[mode]
        L.check(self.lib.sim_set_regions(self.h, m), "sim_set_regions")

    def regions(self, out=None):
        """(region id per cell (device int32, -1 inactive), region count,
        floating-region count) of the current geometry."""
        if out is None:
            out = torch.empty(self.nc, dtype=torch.int32, device="cuda")
        cnt, flo = C.c_int32(0), C.c_int32(0)
        L.check(self.lib.sim_regions(self.h, _ptr(out, self.nc, torch.int32, "regions"), C.byref(cnt),
                                     C.byref(flo), _stream()), "sim_regions")
        return out, cnt.value, flo.value

    def _stats(self, want):
        """(object handed back, pointer passed to the library) for a solver report."""
        if not want:
            return None, None
        if getattr(self, "device_mode", False):
            ds = DeviceStats()
            return ds, ds.ptr()
        st = L.SimStats()
        return st, C.byref(st)

    @staticmethod
    def _report(st):
        if st is None:
            return None
        return st if isinstance(st, DeviceStats) else st.as_dict()

    def _done(self, status, what, st):
        rep = self._report(st)
        L.check(status, what, rep)
        return rep

    def _geom(self, theta, ctrl):
        th, thp = _host_doubles(theta, self.n_params, "theta")
        ct, ctp = _host_doubles(ctrl, self.n_ctrl, "ctrl")
        return (th, ct), thp, ctp

    def step(self, u_n, theta=None, ctrl=None, u_out=None, p_out=None, stats=True):
        f32 = torch.float32
        if u_out is None:
            u_out = torch.empty_like(u_n)
        keep, thp, ctp = self._geom(theta, ctrl)
        st, stp = self._stats(stats)
        rc = self.lib.sim_step(self.h, _ptr(u_n, self.nf, f32, "u_n"), thp, ctp, _ptr(u_out, self.nf, f32, "u_n1"),
                               _ptr(p_out, self.nc, f32, "p_n1"), stp, _stream())
        return u_out, self._done(rc, "sim_step", st)

    def step_replay(self, u_n, p_n1, theta=None, ctrl=None, u_out=None):
        """sim_step with its pressure p_n1 already known (no solve)."""
        f32 = torch.float32
        if u_out is None:
            u_out = torch.empty_like(u_n)
        keep, thp, ctp = self._geom(theta, ctrl)
        L.check(self.lib.sim_step_replay(self.h, _ptr(u_n, self.nf, f32, "u_n"), thp, ctp,
                                         _ptr(p_n1, self.nc, f32, "p_n1"), _ptr(u_out, self.nf, f32, "u_n1"),
                                         _stream()), "sim_step_replay")
        return u_out

    def project(self, u_in, theta=None, ctrl=None, u_out=None, p_out=None, stats=True):
        f32 = torch.float32
        if u_out is None:
            u_out = torch.empty_like(u_in)
        keep, thp, ctp = self._geom(theta, ctrl)
        st, stp = self._stats(stats)
        rc = self.lib.sim_project(self.h, _ptr(u_in, self.nf, f32, "u_in"), thp, ctp,
                                  _ptr(u_out, self.nf, f32, "u_out"), _ptr(p_out, self.nc, f32, "p_out"), stp,
                                  _stream())
        return u_out, self._done(rc, "sim_project", st)

    def step_adjoint(self, u_n, g_u_n1, theta=None, ctrl=None, p_n1=None, g_u_n=None, g_theta=None, g_ctrl=None,
                     stats=True):
        f32, f64 = torch.float32, torch.float64
        if g_u_n is None:
            g_u_n = torch.empty_like(g_u_n1)
        keep, thp, ctp = self._geom(theta, ctrl)
        st, stp = self._stats(stats)
        rc = self.lib.sim_step_adjoint(
            self.h, _ptr(u_n, self.nf, f32, "u_n"), _ptr(p_n1, self.nc, f32, "p_n1"), thp, ctp,
            _ptr(g_u_n1, self.nf, f32, "g_u_n1"), _ptr(g_u_n, self.nf, f32, "g_u_n"),
            _ptr(g_theta, self.n_params, f64, "g_theta") if g_theta is not None else None,
            _ptr(g_ctrl, self.n_ctrl, f64, "g_ctrl") if g_ctrl is not None else None, stp, _stream())
        return g_u_n, self._done(rc, "sim_step_adjoint", st)

    def poisson_solve(self, b, x, alpha=None, tol=0.0, max_iter=0, stats=True):
        f32 = torch.float32
        st, stp = self._stats(stats)
        rc = self.lib.poisson_solve(self.h, _ptr(alpha, self.nf, f32, "alpha"), _ptr(b, self.nc, f32, "b"),
                                    _ptr(x, self.nc, f32, "x"), float(tol), int(max_iter), stp, _stream())
        return x, self._done(rc, "poisson_solve", st)

    def loss_box(self, u, lo=(0.5, 0.5, 0.5), hi=(1.0, 1.0, 1.0), J=None, g=None):
        """J = sum of u^2 over faces centred in [lo, hi] (device double) and g = dJ/du."""
        if J is None:
            J = torch.empty(1, dtype=torch.float64, device=u.device)
        if g is None:
            g = torch.empty_like(u)
        lo_, lop = _host_doubles(lo, 3, "lo")
        hi_, hip = _host_doubles(hi, 3, "hi")
        L.check(self.lib.sim_loss_box(self.h, _ptr(u, self.nf, torch.float32, "u"), lop, hip,
                                      _ptr(J, 1, torch.float64, "J"), _ptr(g, self.nf, torch.float32, "g"),
                                      _stream()), "sim_loss_box")
        return J, g

    def loss_outlet(self, u, scale, w=None, J=None, g=None):
        """J = scale * sum over the outlet faces of w u (device double) and g = dJ/du;
        w: nx * ny outlet weights (device float32) or None for 1."""
        if J is None:
            J = torch.empty(1, dtype=torch.float64, device=u.device)
        if g is None:
            g = torch.empty_like(u)
        nxy = self.cfg.n[0] * self.cfg.n[1]
        L.check(self.lib.sim_loss_outlet(self.h, _ptr(u, self.nf, torch.float32, "u"),
                                         _ptr(w, nxy, torch.float32, "w") if w is not None else None,
                                         float(scale), _ptr(J, 1, torch.float64, "J"),
                                         _ptr(g, self.nf, torch.float32, "g"), _stream()), "sim_loss_outlet")
        return J, g

    def profile(self, kernel):
        """Time every launch of one kernel family with HIP events (None: stop)."""
        kid = -1 if kernel is None else L.KERNELS.index(kernel)
        L.check(self.lib.sim_profile(self.h, kid), "sim_profile")

    def profile_read(self, min_ms=0.0):
        """(total ms, launches) of the timed kernel since the last read, over
        launches that took at least min_ms."""
        ms, cnt = C.c_double(0), C.c_int64(0)
        L.check(self.lib.sim_profile_read(self.h, float(min_ms), C.byref(ms), C.byref(cnt)), "sim_profile_read")
        return ms.value, cnt.value

    def set_geometry(self, theta=None, ctrl=None, alpha_out=None):
        keep, thp, ctp = self._geom(theta, ctrl)
        L.check(self.lib.sim_set_geometry(self.h, thp, ctp, _ptr(alpha_out, self.nf, torch.float32, "alpha"),
                                          _stream()), "sim_set_geometry")
        return alpha_out


# ---- function-style aliases with the C ABI's names -----------------------

def sim_create(cfg: Config) -> Sim:
    return Sim(cfg)


def sim_step(sim: Sim, u_n, theta=None, ctrl=None, u_n1=None, p_n1=None):
    return sim.step(u_n, theta, ctrl, u_n1, p_n1)


def sim_project(sim: Sim, u_in, theta=None, ctrl=None, u_out=None, p_out=None):
    return sim.project(u_in, theta, ctrl, u_out, p_out)


def sim_step_adjoint(sim: Sim, u_n, g_u_n1, theta=None, ctrl=None, p_n1=None, g_u_n=None, g_theta=None,
                     g_ctrl=None):
    return sim.step_adjoint(u_n, g_u_n1, theta, ctrl, p_n1, g_u_n, g_theta, g_ctrl)


def poisson_solve(sim: Sim, b, x, alpha=None, tol=0.0, max_iter=0):
    return sim.poisson_solve(b, x, alpha, tol, max_iter)


def loss_box_noalloc(u, n, dx, lo=(0.5, 0.5, 0.5), hi=(1.0, 1.0, 1.0), J=None, g=None):
    """The box loss without a handle (the library allocates nothing): J = sum
    of u^2 over faces centred in [lo, hi] (device double) and g = dJ/du on an
    n = (nx, ny, nz) grid of cell width dx."""
    lib = L.load()
    n = tuple(int(v) for v in n)
    nx, ny, nz = n
    nf = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    if J is None:
        J = torch.empty(1, dtype=torch.float64, device=u.device)
    if g is None:
        g = torch.empty_like(u)
    n_ = (C.c_int32 * 3)(*n)
    lo_, lop = _host_doubles(lo, 3, "lo")
    hi_, hip = _host_doubles(hi, 3, "hi")
    L.check(lib.sim_loss_box_noalloc(n_, float(dx), _ptr(u, nf, torch.float32, "u"), lop, hip,
                                     _ptr(J, 1, torch.float64, "J"), _ptr(g, nf, torch.float32, "g"), _stream()),
            "sim_loss_box_noalloc")
    return J, g


def ellipsoid_poses(theta0, ctrl, dt) -> np.ndarray:
    """(T, 15) per-step ellipsoid geometry (c, a, R) from theta0 (9) and ctrl (T, 6)."""
    lib = L.load()
    th = np.ascontiguousarray(np.asarray(theta0, np.float64).ravel())
    ct = np.ascontiguousarray(np.asarray(ctrl, np.float64).reshape(-1, 6))
    if th.size != 9:
        raise ValueError("theta0 must hold 9 values")
    T = ct.shape[0]
    out = np.zeros((T, 15))
    dp = C.POINTER(C.c_double)
    L.check(lib.sim_ellipsoid_poses(th.ctypes.data_as(dp), ct.ctypes.data_as(dp), T, float(dt),
                                    out.ctypes.data_as(dp)), "sim_ellipsoid_poses")
    return out


def ellipsoid_poses_adjoint(theta0, ctrl, dt, g_steps, g_ctrl_direct):
    """Chain per-step partials through the pose dynamics: returns (dJ/dtheta0 (9), dJ/dctrl (T, 6))."""
    lib = L.load()
    th = np.ascontiguousarray(np.asarray(theta0, np.float64).ravel())
    ct = np.ascontiguousarray(np.asarray(ctrl, np.float64).reshape(-1, 6))
    T = ct.shape[0]
    gs = np.ascontiguousarray(np.asarray(g_steps, np.float64).reshape(T, 15))
    gd = np.ascontiguousarray(np.asarray(g_ctrl_direct, np.float64).reshape(T, 6))
    gth = np.zeros(9)
    gct = np.zeros((T, 6))
    dp = C.POINTER(C.c_double)
    L.check(lib.sim_ellipsoid_poses_adjoint(th.ctypes.data_as(dp), ct.ctypes.data_as(dp), T, float(dt),
                                            gs.ctypes.data_as(dp), gd.ctypes.data_as(dp),
                                            gth.ctypes.data_as(dp), gct.ctypes.data_as(dp)),
            "sim_ellipsoid_poses_adjoint")
    return gth, gct
