"""Continuous-batching serving loop for rollout and Poisson-projection requests.

Requests arrive over time (Poisson arrivals), each with its own grid size,
step count, mode (forward only, forward + adjoint, or one pressure
projection) and seeded scene.  A request is admitted as soon as its device
footprint (the library's workspace, from ``sim_footprint``, plus its episode
tensors) fits in the remaining HBM budget and a concurrency slot is free; it
then runs on its own HIP stream, driven by its own host thread (the library
releases the GIL inside every call), so the kernels of all admitted episodes
overlap on the GPU.  Library handles are pooled per configuration, so an
admitted request reuses a warm workspace.  When an episode completes its
memory and slot are freed and the queue is re-examined.  Results and per-step
latencies are kept per request.

Inputs are generated on the device from each request's seed (a vector
potential drawn with torch's generator, blurred and curled): they are input
plumbing, not the method, and are produced before the request's timed steps.
"""
from __future__ import annotations

import heapq
import math
import threading
import time
from collections import defaultdict, deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .sim import Config, Sim, sim_footprint, ellipsoid_poses


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the stream
    n: int                    # cells per axis (cubic grid)
    steps: int
    mode: str                 # "fwd" | "fwd+adj" | "poisson"
    seed: int
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    step_ms: list = field(default_factory=list)
    result: dict = field(default_factory=dict)
    error: str = ""


def make_stream(count, rate, seed=0, sizes=(32, 48, 64, 96, 128, 192), steps=(8, 64), kinds=("fwd", "fwd+adj")):
    """Seeded request stream: exponential inter-arrival times at `rate` req/s,
    grid size uniform over `sizes`, steps uniform in [steps[0], steps[1]],
    mode uniform over `kinds`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        out.append(Request(i, t, int(rng.choice(sizes)), int(rng.integers(steps[0], steps[1] + 1)),
                           str(rng.choice(kinds)), int(seed * 100003 + i)))
    return out


# ---------------------------------------------------------------------------
# device-side scene inputs (plumbing)
# ---------------------------------------------------------------------------

def _blur_axis(x, k, dim):
    # taps summed in a fixed order with elementwise ops: the same bits whatever
    # else runs on the device (a library convolution may pick its algorithm,
    # and so its rounding, by the workspace memory it finds free)
    r = (k.numel() - 1) // 2
    xs = torch.movedim(x, dim, -1)
    shp = xs.shape
    m = shp[-1]
    xp = torch.nn.functional.pad(xs.reshape(-1, 1, m), (r, r), mode="reflect").reshape(-1, m + 2 * r)
    y = k[0] * xp[:, 0:m]
    for t in range(1, 2 * r + 1):
        y = y + k[t] * xp[:, t:t + m]
    return torch.movedim(y.reshape(shp), -1, dim)


def device_curl_noise(n, seed, device="cuda", sigma=2.0):
    """Divergence-free random face velocity (canonical layout, max |u| = 1)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = int(math.ceil(4 * sigma))
    xs = torch.arange(-r, r + 1, device=device, dtype=torch.float32)
    k = torch.exp(-0.5 * (xs / sigma) ** 2)
    k = k / k.sum()

    def field(shape):
        a = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
        for dim in range(3):
            if a.shape[dim] > r:
                a = _blur_axis(a, k, dim)
        return a
    psx = field((n + 1, n + 1, n))
    psy = field((n + 1, n, n + 1))
    psz = field((n, n + 1, n + 1))
    psy[:, :, 0] = 0; psy[:, :, -1] = 0; psz[:, :, 0] = 0; psz[:, :, -1] = 0
    psx[:, 0, :] = 0; psx[:, -1, :] = 0; psz[:, 0, :] = 0; psz[:, -1, :] = 0
    psx[0] = 0; psx[-1] = 0; psy[0] = 0; psy[-1] = 0
    ux = (psz[:, 1:, :] - psz[:, :-1, :]) - (psy[1:, :, :] - psy[:-1, :, :])
    uy = (psx[1:, :, :] - psx[:-1, :, :]) - (psz[:, :, 1:] - psz[:, :, :-1])
    uz = (psy[:, :, 1:] - psy[:, :, :-1]) - (psx[:, 1:, :] - psx[:, :-1, :])
    u = torch.cat([ux.reshape(-1), uy.reshape(-1), uz.reshape(-1)])
    return (u / u.abs().max()).contiguous()


def request_scene(req: Request):
    rng = np.random.default_rng(req.seed)
    c = rng.uniform(0.35, 0.65, 3)
    a = rng.uniform(0.08, 0.2, 3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    theta0 = np.concatenate([c, a, d * math.pi * rng.uniform() ** (1 / 3)])
    ctrl = rng.uniform(-0.5, 0.5, (max(req.steps, 1), 6))
    return theta0, ctrl


# ---------------------------------------------------------------------------
# one episode
# ---------------------------------------------------------------------------

def episode_bytes(n, steps, mode, every=8):
    nf = 3 * (n + 1) * n * n
    per = 4 * nf
    if mode == "fwd+adj":
        k = max(1, min(every, steps))
        return per * (steps // every + 2 + (k + 1) + 3) + 4 * n ** 3 * k
    return per * 3


def run_episode(sim: Sim, req: Request, stream, timing=True, every=8):
    """Run one request on `stream` with handle `sim`; fills req.result / step_ms."""
    from .rollout import Rollout
    with torch.cuda.stream(stream):
        theta0, ctrl = request_scene(req)
        u0 = device_curl_noise(req.n, req.seed)
        if req.mode == "poisson":
            poses = ellipsoid_poses(theta0, ctrl[:1], sim.cfg.dt)
            t0 = time.perf_counter()
            out, st = sim.project(u0, poses[0], ctrl[0])
            stream.synchronize()
            req.step_ms.append(1e3 * (time.perf_counter() - t0))
            req.result = {"u": out, "iters": st["iters"]}
            return
        timer = _HostTimer(req.step_ms, stream) if timing else None
        ro = Rollout.ellipsoid(sim, theta0, ctrl[:req.steps], every=every, timer=timer)
        uT = ro.forward(u0)
        req.result = {"u": uT}
        if req.mode == "fwd+adj":
            J, g = sim.loss_box(uT)
            g0 = ro.backward(g)
            gth, gct = ro.geometry_gradients()
            req.result.update({"g_u0": g0, "g_theta0": gth, "g_ctrl": gct, "loss": J})
        stream.synchronize()


class _HostTimer:
    """Per-step wall latency (each library step ends with a stream-synchronised
    convergence check, so host time brackets the step's device work)."""

    def __init__(self, sink, stream):
        self.sink, self.stream, self.t = sink, stream, 0.0

    def begin(self, kind):
        self.t = time.perf_counter()

    def end(self, kind):
        self.stream.synchronize()
        self.sink.append(1e3 * (time.perf_counter() - self.t))


# ---------------------------------------------------------------------------
# admission and the serving loop
# ---------------------------------------------------------------------------

class Admission:
    """HBM-footprint admission: FIFO queue, admit while the budget and the
    slot count allow; a request larger than the whole budget is rejected."""

    def __init__(self, budget_bytes, max_active, footprint):
        self.budget, self.max_active, self.footprint = budget_bytes, max_active, footprint
        self.queue = deque()
        self.used = 0
        self.active = {}

    def offer(self, req):
        need = self.footprint(req)
        if need > self.budget:
            req.error = f"needs {need} B > budget {self.budget} B"
            return False
        self.queue.append((req, need))
        return True

    def admit(self):
        out = []
        while self.queue and len(self.active) < self.max_active and self.used + self.queue[0][1] <= self.budget:
            req, need = self.queue.popleft()
            self.used += need
            self.active[req.rid] = need
            out.append(req)
        return out

    def release(self, req):
        self.used -= self.active.pop(req.rid)


class HandlePool:
    """Warm library handles keyed by (grid, precision)."""

    def __init__(self, precision, tol=1e-6):
        self.precision, self.tol = precision, tol
        self.free = defaultdict(list)
        self.lock = threading.Lock()

    def cfg(self, n):
        return Config(n=(n, n, n), dx=1.0 / n, dt=0.5 / n, geom="ellipsoid", tol=self.tol,
                      precision=self.precision, max_iter=200)

    def get(self, n):
        with self.lock:
            if self.free[n]:
                return self.free[n].pop()
        return Sim(self.cfg(n))

    def put(self, n, sim):
        with self.lock:
            self.free[n].append(sim)

    def close(self):
        for lst in self.free.values():
            for s in lst:
                s.close()
        self.free.clear()


def serve(requests, budget_bytes, precision="fp16", max_active=8, realtime=True, timing=True, on_done=None):
    """Run the stream with continuous batching.  Returns a summary dict.
    on_done(req), if given, is called from the loop as each request completes."""
    pool = HandlePool(precision)
    adm = Admission(budget_bytes, max_active,
                    lambda r: sim_footprint(pool.cfg(r.n)) + episode_bytes(r.n, r.steps, r.mode))
    done_q = deque()
    cv = threading.Condition()
    pending = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()

    def worker(req):
        sim = pool.get(req.n)
        stream = torch.cuda.Stream()
        try:
            req.admitted = time.perf_counter() - t0
            run_episode(sim, req, stream, timing)
        except Exception as e:  # a failing request is reported, the others go on
            req.error = repr(e)
        finally:
            req.finished = time.perf_counter() - t0
            pool.put(req.n, sim)
            with cv:
                done_q.append(req)
                cv.notify()

    threads = []
    i = 0
    finished = 0
    total = len(pending)
    rejected = []
    while finished + len(rejected) < total:
        now = time.perf_counter() - t0
        while i < total and (not realtime or pending[i].arrival <= now):
            if not adm.offer(pending[i]):
                rejected.append(pending[i])
            i += 1
        for req in adm.admit():
            th = threading.Thread(target=worker, args=(req,), daemon=True)
            th.start()
            threads.append(th)
        with cv:
            if not done_q:
                wait = 0.05
                if realtime and i < total:
                    wait = max(0.0, min(wait, pending[i].arrival - (time.perf_counter() - t0)))
                cv.wait(timeout=wait)
            while done_q:
                r = done_q.popleft()
                adm.release(r)
                finished += 1
                if on_done:
                    on_done(r)
    for th in threads:
        th.join()
    wall = time.perf_counter() - t0
    torch.cuda.synchronize()
    pool.close()
    return summarize(requests, wall, rejected)


def serve_serial(requests, precision="fp32", timing=True, on_done=None):
    """Baseline: one request at a time, FIFO, in arrival order (no overlap)."""
    pool = HandlePool(precision)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r.arrival):
        sim = pool.get(req.n)
        req.admitted = time.perf_counter() - t0
        try:
            run_episode(sim, req, stream, timing)
        except Exception as e:
            req.error = repr(e)
        req.finished = time.perf_counter() - t0
        pool.put(req.n, sim)
        if on_done:
            on_done(req)
    wall = time.perf_counter() - t0
    pool.close()
    return summarize(requests, wall, [])


def summarize(requests, wall, rejected):
    ok = [r for r in requests if not r.error]
    steps = [ms for r in ok for ms in r.step_ms]
    # every step counts once (a forward step and its adjoint are one cell-step,
    # as in the rollout benchmark); a projection request counts as one step
    cell_steps = 0
    for r in ok:
        cell_steps += r.n ** 3 * (1 if r.mode == "poisson" else r.steps)
    lat = [r.finished - r.arrival for r in ok if not math.isnan(r.finished)]

    def p(v, q):
        if not v:
            return None
        s = sorted(v)
        return s[min(len(s) - 1, max(0, int(math.ceil(q / 100 * len(s))) - 1))]
    return {"requests": len(requests), "completed": len(ok), "rejected": len(rejected),
            "failed": sum(1 for r in requests if r.error) - len(rejected),
            "wall_s": wall, "cell_steps_per_s": cell_steps / wall if wall > 0 else 0.0,
            "step_ms_p50": p(steps, 50), "step_ms_p99": p(steps, 99),
            "request_s_p50": p(lat, 50), "request_s_p99": p(lat, 99)}
