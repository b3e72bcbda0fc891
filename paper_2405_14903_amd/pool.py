"""The library's serving pool (``sim_pool_*`` in include/neuralfluid.h): many
episodes at once, each on a handle and a stream of its own, advanced one unit
per tick, admitted by HBM footprint.  This module only marshals arguments.

Episode kinds: ``"fwd"`` (T forward steps, result u_T), ``"fwd+adj"`` (the
same, then the box loss of u_T and the full adjoint: dJ/du_0 and the per-step
dJ/dtheta, dJ/dctrl) and ``"poisson"`` (one pressure projection of u_0).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from .sim import Config, _host_doubles, _ptr

_KIND = {"fwd": L.SIM_EP_FORWARD, "fwd+adj": L.SIM_EP_FORWARD_ADJOINT, "poisson": L.SIM_EP_PROJECT}


class Pool:
    """``Pool(budget_bytes, max_active, inflight_cells)``; ``admit`` returns a
    slot (None when the pool is busy: no free slot or budget), ``tick``
    enqueues the next unit of every active episode the in-flight bounds allow
    (waiting for the oldest unit in flight when none could be enqueued) and
    returns how many still have work to enqueue, ``poll`` tells whether a
    slot's work has completed, ``result`` collects it and frees the slot.
    inflight_cells bounds the grid cells of the units in flight (0: no bound
    beyond two units per episode)."""

    def __init__(self, budget_bytes: int, max_active: int = 8, inflight_cells: int = 0):
        self.lib = L.load()
        self.h = C.c_void_p()
        L.check(self.lib.sim_pool_create(int(budget_bytes), int(max_active), int(inflight_cells), C.byref(self.h)),
                "sim_pool_create")
        self.episodes = {}

    def close(self):
        if self.h:
            L.check(self.lib.sim_pool_destroy(self.h), "sim_pool_destroy")
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def admit(self, cfg: Config, kind: str, u0: torch.Tensor, theta=None, ctrl=None, steps: int = 1, every: int = 8,
              box=((0.5, 0.5, 0.5), (1.0, 1.0, 1.0)), host_checked: bool = False):
        """host_checked: every solve waits for its convergence state, whatever
        budget the grid has learned (to rerun an episode whose device-mode
        solve missed the tolerance; that also doubled the grid's budget)."""
        d = cfg.desc()
        T = 1 if kind == "poisson" else int(steps)
        ep = L.SimEpisode()
        ep.desc = d
        ep.kind = _KIND[kind]
        ep.steps = T
        ep.every = int(every)
        ep.flags = L.SIM_EP_HOST_CHECKED if host_checked else 0
        th, thp = _host_doubles(theta, T * d.n_params, "theta")
        ct, ctp = _host_doubles(ctrl, T * d.n_ctrl, "ctrl")
        ep.theta, ep.ctrl = thp, ctp
        for a in range(3):
            ep.box_lo[a], ep.box_hi[a] = float(box[0][a]), float(box[1][a])
        nf = cfg.nfaces
        # the pool's copy runs on its own stream: u0 must be complete
        torch.cuda.current_stream().synchronize()
        slot = C.c_int32(-1)
        rc = self.lib.sim_pool_admit(self.h, C.byref(ep), _ptr(u0, nf, torch.float32, "u0"), C.byref(slot))
        if rc == L.SIM_EBUSY:
            return None
        L.check(rc, "sim_pool_admit")
        # u0 is read on the pool's stream: keep it alive until the result
        self.episodes[slot.value] = (cfg, kind, T, d.n_params, d.n_ctrl, u0)
        return slot.value

    def tick(self) -> int:
        pending = C.c_int32(0)
        L.check(self.lib.sim_pool_tick(self.h, C.byref(pending)), "sim_pool_tick")
        return pending.value

    def poll(self, slot: int) -> bool:
        done = C.c_int32(0)
        L.check(self.lib.sim_pool_poll(self.h, int(slot), C.byref(done)), "sim_pool_poll")
        return bool(done.value)

    def result(self, slot: int, want_u: bool = True, raise_on_warning: bool = False):
        """dict(u, g_u0, g_theta (T, n_params) or None, g_ctrl (T, n_ctrl) or
        None, J, worst (the solves summarised), status)."""
        cfg, kind, T, npar, nctl, _u0 = self.episodes.pop(slot)
        dev = torch.device("cuda")
        nf = cfg.nfaces
        u = torch.empty(nf, dtype=torch.float32, device=dev) if want_u else None
        adj = kind == "fwd+adj"
        gu = torch.empty(nf, dtype=torch.float32, device=dev) if adj else None
        gth = torch.zeros((T, npar), dtype=torch.float64, device=dev) if adj and npar else None
        gct = torch.zeros((T, nctl), dtype=torch.float64, device=dev) if adj and nctl else None
        J = C.c_double(0.0)
        worst = L.SimStats()
        # the copies run on the pool's stream: the outputs' memory must not
        # still be in use by work on the current stream
        torch.cuda.current_stream().synchronize()
        rc = self.lib.sim_pool_result(self.h, int(slot), _ptr(u, nf, torch.float32, "u"),
                                      _ptr(gu, nf, torch.float32, "g_u0"),
                                      C.c_void_p(gth.data_ptr()) if gth is not None else None,
                                      C.c_void_p(gct.data_ptr()) if gct is not None else None,
                                      C.byref(J), C.byref(worst))
        if rc < 0 or (raise_on_warning and rc > 0):
            L.check(rc, "sim_pool_result", worst.as_dict())
        return {"u": u, "g_u0": gu, "g_theta": gth, "g_ctrl": gct, "J": J.value if adj else None,
                "worst": worst.as_dict(), "status": rc}

    def run(self, jobs):
        """Admit `jobs` (dicts of admit's keyword arguments) in order as slots
        and budget free up, and tick until every one is done; returns their
        results in job order."""
        queue = list(enumerate(jobs))
        live, out = {}, [None] * len(queue)
        retry = True                       # admission can succeed (a slot or memory was released)
        while queue or live:
            while queue and retry:
                i, job = queue[0]
                s = self.admit(**job)
                if s is None:
                    if not live:
                        raise RuntimeError("an episode does not fit the pool's budget even when the pool is empty")
                    retry = False
                    break
                live[s] = i
                queue.pop(0)
            self.tick()
            for s in [s for s in live if self.poll(s)]:
                out[live.pop(s)] = self.result(s)
                retry = True
        return out
