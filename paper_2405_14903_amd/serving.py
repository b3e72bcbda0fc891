"""Continuous-batching serving loop for rollout and Poisson-projection requests.

Requests arrive over time (Poisson arrivals), each with its own grid size,
step count, mode (forward only, forward + adjoint, or one pressure
projection) and seeded scene.  A request is admitted as soon as its device
memory fits in the HBM budget (every library handle, busy or idle, counts
with its ``sim_footprint``, plus the episode's own tensors; idle handles are
freed least recently used first when a request needs the room) and a slot is
free.  Each admitted episode gets its own HIP stream and runs with the
library's device solve mode, so no call waits on the host: one host thread
enqueues the episodes' steps round-robin, one step of an episode at a time,
and keeps at most two steps of each episode and a bounded number of grid
cells in flight, so that the kernels of small episodes overlap with each
other and with one large one while a large step never queues behind many
others.  Completion is polled with events.  Per-step latencies come from
event pairs around each step on its episode's stream; the solver reports of
every step are read when the episode has finished, and a step whose solve
missed the tolerance makes its request fail.

The serial baseline runs the same requests one at a time, each starting no
earlier than its arrival, with the plain host-checked FP32 path.

Inputs are generated on the device from each request's seed (a vector
potential drawn with torch's generator, blurred and curled): they are input
plumbing, not the method, and are produced before the request's first step.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
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


def make_stream(count, rate, seed=0, sizes=(32, 48, 64, 96, 128, 192), steps=(8, 64), poisson_share=0.1):
    """Seeded request stream: exponential inter-arrival times at `rate` req/s,
    grid size uniform over `sizes`, steps uniform in [steps[0], steps[1]];
    a share `poisson_share` of the requests are single pressure projections,
    the rest half forward-only and half forward + adjoint rollouts."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        st = int(rng.integers(steps[0], steps[1] + 1))
        u = rng.uniform()
        mode = "poisson" if u < poisson_share else ("fwd" if u < poisson_share + 0.5 * (1 - poisson_share)
                                                    else "fwd+adj")
        out.append(Request(i, t, n, st, mode, int(seed * 100003 + i)))
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
    """Device bytes of one episode's own tensors: velocity fields (input,
    state pair, checkpoints, segment states, gradients) and, for forward +
    adjoint, the pressure of every step kept by the first forward."""
    nf = 3 * (n + 1) * n * n
    per = 4 * nf
    if mode == "fwd+adj":
        k = max(1, min(every, steps))
        return per * (steps // every + 2 + (k + 1) + 3) + 4 * n ** 3 * steps
    return per * 3


def episode_steps(sim: Sim, req: Request, every=8, stats_sink=None):
    """The work of one request as a generator: each `next` enqueues one unit
    (the input set-up, then one forward, recomputed or adjoint step, or the
    projection) on the current stream and yields its kind.  Results are
    left as device tensors in req.result; the shape and control gradients
    need a host read and are formed by :func:`finish_episode` once the work
    has run."""
    from .rollout import Rollout
    theta0, ctrl = request_scene(req)
    u0 = device_curl_noise(req.n, req.seed)
    if req.mode == "poisson":
        yield "setup"
        poses = ellipsoid_poses(theta0, ctrl[:1], sim.cfg.dt)
        out, st = sim.project(u0, poses[0], ctrl[0], stats=stats_sink is not None)
        if stats_sink is not None:
            stats_sink.append(("fwd", st))
        req.result = {"u": out}
        yield "poisson"
        return
    yield "setup"
    ro = Rollout.ellipsoid(sim, theta0, ctrl[:req.steps], every=every, store_pressure=req.mode == "fwd+adj")
    if stats_sink is not None:
        ro.device_stats = stats_sink
    yield from ro.forward_steps(u0)
    req.result = {"u": ro.uT}
    if req.mode == "fwd+adj":
        J, g = sim.loss_box(ro.uT)
        yield from ro.backward_steps(g)
        req.result.update({"g_u0": ro.g0, "loss": J, "_rollout": ro})


def finish_episode(req: Request):
    """Host-side end of a finished episode (its stream has reached its end)."""
    ro = req.result.pop("_rollout", None)
    if ro is not None:
        gth, gct = ro.geometry_gradients()
        req.result.update({"g_theta0": gth, "g_ctrl": gct})


def run_episode(sim: Sim, req: Request, stream, timing=True, every=8):
    """Run one request to its end on `stream` (its steps back to back); per-
    step latencies from event pairs on the stream."""
    with torch.cuda.stream(stream):
        marks = []
        for kind in _timed(episode_steps(sim, req, every), marks, timing):
            pass
        stream.synchronize()
    req.step_ms += [a.elapsed_time(b) for a, b, k in marks if k != "setup"]
    finish_episode(req)


def _timed(gen, marks, timing):
    """Bracket each unit of a generator with events on the current stream."""
    while True:
        a = torch.cuda.Event(enable_timing=True) if timing else None
        if a is not None:
            a.record()
        try:
            kind = next(gen)
        except StopIteration:
            return
        if a is not None:
            b = torch.cuda.Event(enable_timing=True)
            b.record()
            marks.append((a, b, kind))
        yield kind


# ---------------------------------------------------------------------------
# admission and handles
# ---------------------------------------------------------------------------

class Admission:
    """HBM-footprint admission with pooled library handles.

    Every live handle, busy or idle, counts with its workspace bytes; an
    admitted request adds its episode bytes.  The queue is FIFO: the head is
    admitted when a slot is free and its bytes fit (reusing an idle handle of
    its grid, whose bytes are already counted, or creating one), after
    freeing idle handles of other grids least recently used first if that
    makes it fit.  A request that could not fit even in an empty server is
    rejected when offered.

    handle_bytes(n) -> workspace bytes of a handle for grid n;
    episode_bytes(req) -> the request's own device bytes;
    make(n) -> a new handle (with .close())."""

    def __init__(self, budget_bytes, max_active, handle_bytes, episode_bytes, make):
        self.budget, self.max_active = budget_bytes, max_active
        self.handle_bytes, self.episode_bytes, self.make = handle_bytes, episode_bytes, make
        self.queue = deque()
        self.used = 0                 # live handles + active episodes
        self.active = {}              # rid -> (episode bytes, grid)
        self.idle = OrderedDict()     # (grid, serial) -> handle, least recently used first
        self._serial = 0

    def offer(self, req):
        need = self.handle_bytes(req.n) + self.episode_bytes(req)
        if need > self.budget:
            req.error = f"needs {need} B > budget {self.budget} B"
            return False
        self.queue.append(req)
        return True

    def _idle_for(self, n):
        for key in self.idle:
            if key[0] == n:
                return key
        return None

    def admit(self):
        """[(request, handle)] admitted now, in FIFO order."""
        out = []
        while self.queue and len(self.active) < self.max_active:
            req = self.queue[0]
            ep = self.episode_bytes(req)
            key = self._idle_for(req.n)
            need = ep if key is not None else ep + self.handle_bytes(req.n)
            # free idle handles of other grids, least recently used first
            while self.used + need > self.budget:
                victim = next((k for k in self.idle if k != key), None)
                if victim is None:
                    break
                self.idle.pop(victim).close()
                self.used -= self.handle_bytes(victim[0])
            if self.used + need > self.budget:
                break
            self.queue.popleft()
            if key is not None:
                h = self.idle.pop(key)
            else:
                h = self.make(req.n)
            self.used += need
            self.active[req.rid] = (ep, req.n)
            out.append((req, h))
        return out

    def release(self, req, handle):
        """The request is done: its episode bytes are freed and its handle
        goes idle (still counted)."""
        ep, n = self.active.pop(req.rid)
        self.used -= ep
        self._serial += 1
        self.idle[(n, self._serial)] = handle

    def warm(self, n):
        """Create an idle handle for grid n up front (counted); False if it
        does not fit."""
        if self.used + self.handle_bytes(n) > self.budget:
            return False
        self._serial += 1
        self.idle[(n, self._serial)] = self.make(n)
        self.used += self.handle_bytes(n)
        return True

    def close(self):
        for h in self.idle.values():
            h.close()
        for key in list(self.idle):
            self.used -= self.handle_bytes(key[0])
        self.idle.clear()


def handle_config(n, precision, tol=1e-6):
    return Config(n=(n, n, n), dx=1.0 / n, dt=0.5 / n, geom="ellipsoid", tol=tol, precision=precision, max_iter=200)


# ---------------------------------------------------------------------------
# the serving loop
# ---------------------------------------------------------------------------

class _Episode:
    def __init__(self, req, sim, timing):
        self.req, self.sim = req, sim
        self.stream = torch.cuda.Stream()
        self.stats = []
        with torch.cuda.stream(self.stream):
            self.gen = episode_steps(sim, req, stats_sink=self.stats)
        self.marks = deque()          # (start, end, kind) of steps in flight
        self.timing = timing
        self.exhausted = False
        self.last = None              # event after the latest enqueued step

    def advance(self):
        with torch.cuda.stream(self.stream):
            a = torch.cuda.Event(enable_timing=self.timing)
            a.record()
            try:
                kind = next(self.gen)
            except StopIteration:
                self.exhausted = True
                return False
            b = torch.cuda.Event(enable_timing=self.timing)
            b.record()
        self.marks.append((a, b, kind))
        self.last = b
        return True

    def retire(self):
        """Steps that have run: their latencies (ms)."""
        while self.marks and self.marks[0][1].query():
            a, b, kind = self.marks.popleft()
            if self.timing and kind != "setup":
                self.req.step_ms.append(a.elapsed_time(b))

    def finished(self):
        return self.exhausted and not self.marks


def warm_up(sim, n):
    """One short rollout on a fresh handle with host-checked solves (its
    iteration graphs are captured and its kernels loaded before the clock
    starts).  Returns the most CG iterations a solve took."""
    from .rollout import Rollout
    mode = getattr(sim, "device_mode", False)
    sim.set_solve_mode("host")
    req = Request(-1, 0.0, n, 2, "fwd+adj", 7)
    theta0, ctrl = request_scene(req)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        u0 = device_curl_noise(n, req.seed)
        ro = Rollout.ellipsoid(sim, theta0, ctrl[:2], every=8)
        J, g = sim.loss_box(ro.forward(u0))
        ro.backward(g)
    stream.synchronize()
    if mode:
        sim.set_solve_mode("device", getattr(sim, "budget", 0))
    return max(ro.iters["fwd"] + ro.iters["adj"] + [1])


def device_budget(iters):
    """Iteration budget of a device-mode solve from the iterations such solves
    took: half as many again plus two, in whole check intervals of 8."""
    return int(8 * math.ceil((1.5 * iters + 2) / 8))


def serve(requests, budget_bytes, precision="fp16", max_active=8, realtime=True, timing=True, on_done=None,
          inflight_cells=2 * 192 ** 3, solve_budget=0, warm_sizes=()):
    """Run the stream with continuous batching.  Returns a summary dict.
    on_done(req), if given, is called from the loop as each request ends.
    inflight_cells bounds the grid cells of the steps enqueued at once (one
    step may always run); solve_budget is the CG iteration budget of every
    device-mode solve (0: per grid, from the iterations a warm-up rollout's
    host-checked solves took; a request with a solve that missed the
    tolerance is run again with host-checked solves and doubles its grid's
    budget); warm_sizes: grids that get a warmed idle handle before the clock
    starts (counted in the budget like any other)."""
    budget_for = {}      # grid -> device-mode iteration budget, learned from warm-up and from failures

    def make(n):
        sim = Sim(handle_config(n, precision))
        if n not in budget_for:
            budget_for[n] = device_budget(warm_up(sim, n)) if solve_budget <= 0 else solve_budget
        sim.budget = budget_for[n]
        sim.set_solve_mode("device", sim.budget)
        return sim
    adm = Admission(budget_bytes, max_active, lambda n: sim_footprint(handle_config(n, precision)),
                    lambda r: episode_bytes(r.n, r.steps, r.mode), make)
    for n in warm_sizes:
        adm.warm(n)
    pending = sorted(requests, key=lambda r: r.arrival)
    active = []
    rejected = []
    i = finished = 0
    total = len(pending)
    rr = 0
    t0 = time.perf_counter()
    while finished + len(rejected) < total:
        now = time.perf_counter() - t0
        while i < total and (not realtime or pending[i].arrival <= now):
            if not adm.offer(pending[i]):
                rejected.append(pending[i])
            i += 1
        for req, sim in adm.admit():
            req.admitted = time.perf_counter() - t0
            try:
                active.append(_Episode(req, sim, timing))
            except Exception as e:  # a request that cannot start is reported, the others go on
                req.error = repr(e)
                req.finished = req.admitted
                adm.release(req, sim)
                finished += 1
        progressed = False
        cells = sum(ep.req.n ** 3 * len(ep.marks) for ep in active)
        m = len(active)
        for q in range(m):
            ep = active[(rr + q) % m]
            ep.retire()
            if ep.exhausted or len(ep.marks) >= 2:
                continue
            c = ep.req.n ** 3
            if cells > 0 and cells + c > inflight_cells:
                continue
            try:
                if ep.advance():
                    cells += c
                    progressed = True
            except Exception as e:
                ep.req.error = repr(e)
                ep.exhausted = True
        rr += 1
        for ep in [e for e in active if e.finished() or (e.req.error and not e.marks)]:
            active.remove(ep)
            req = ep.req
            ep.stream.synchronize()
            req.finished = time.perf_counter() - t0
            if not req.error:
                try:
                    bad = [k for k, st in ep.stats if not st.as_dict()["converged"]]
                    if bad:
                        # the budget was too small: run the request again with
                        # host-checked solves, and give its grid more
                        budget_for[req.n] = 2 * ep.sim.budget
                        ep.sim.budget = budget_for[req.n]
                        ep.sim.set_solve_mode("host")
                        req.result, req.step_ms = {}, []
                        req.retried = len(bad)
                        run_episode(ep.sim, req, ep.stream)
                        ep.sim.set_solve_mode("device", ep.sim.budget)
                    else:
                        finish_episode(req)
                except Exception as e:
                    req.error = repr(e)
            adm.release(req, ep.sim)
            finished += 1
            progressed = True
            if on_done:
                on_done(req)
        if not progressed:
            # nothing could be enqueued: wait for the oldest step in flight, or
            # for the next arrival
            waits = [ep.marks[0][1] for ep in active if ep.marks]
            if waits:
                waits[0].synchronize()
            elif realtime and i < total:
                time.sleep(max(0.0, min(0.05, pending[i].arrival - (time.perf_counter() - t0))))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    adm.close()
    return summarize(requests, wall, rejected)


def serve_serial(requests, precision="fp32", timing=True, on_done=None, realtime=True, warm_sizes=()):
    """Baseline: one request at a time in arrival order, each starting no
    earlier than its arrival (the same schedule as :func:`serve`), with the
    plain host-checked solves."""
    pool = {}
    for n in warm_sizes:
        pool[n] = Sim(handle_config(n, precision))
        warm_up(pool[n], n)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r.arrival):
        if realtime:
            wait = req.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
        sim = pool.get(req.n)
        if sim is None:
            sim = pool[req.n] = Sim(handle_config(req.n, precision))
        req.admitted = time.perf_counter() - t0
        try:
            run_episode(sim, req, stream, timing)
        except Exception as e:
            req.error = repr(e)
        req.finished = time.perf_counter() - t0
        if on_done:
            on_done(req)
    wall = time.perf_counter() - t0
    for sim in pool.values():
        sim.close()
    return summarize(requests, wall, [])


def serve_pool(requests, budget_bytes, precision="fp16", max_active=8, realtime=True, warm_sizes=(),
               on_done=None, every=8, inflight_cells=2 * 192 ** 3):
    """The same request stream through the library's native pool
    (:class:`paper_2405_14903_amd.pool.Pool`: admission by footprint, one
    unit of every active episode per tick within the in-flight bounds,
    device-mode solves after a grid's first episode).  Requests are admitted
    no earlier than their arrival and in arrival order; one whose footprint
    does not fit waits until a result has released capacity.  A request
    whose device-mode solve missed the tolerance (the pool then doubles its
    grid's budget) is run again at once with host-checked solves, as the
    Python scheduler does.  The pool reports whole requests, so step
    latencies are not measured."""
    from . import _lib as L
    from .pool import Pool
    from .sim import ellipsoid_poses

    def job(req):
        theta0, ctrl = request_scene(req)
        T = 1 if req.mode == "poisson" else req.steps
        poses = ellipsoid_poses(theta0, ctrl[:T], 0.5 / req.n)
        return dict(cfg=handle_config(req.n, precision), kind=req.mode, u0=device_curl_noise(req.n, req.seed),
                    theta=np.asarray(poses)[:T], ctrl=ctrl[:T], steps=T, every=every)

    pool = Pool(budget_bytes, max_active, inflight_cells)
    try:
        # each grid's first episode runs host-checked and sets its iteration
        # budget: do that before the clock starts (the kernels load then too)
        warm = [Request(-1 - i, 0.0, n, 2, "fwd+adj", 7) for i, n in enumerate(warm_sizes)]
        if warm:
            pool.run([job(r) for r in warm])
        queue = sorted(requests, key=lambda r: r.arrival)
        live = {}
        head = None                  # the admission arguments of queue[0], built once
        rerun = []                   # requests to run again host-checked, before the queue
        retry = True                 # the head may fit (a result released capacity since it last did not)
        t0 = time.perf_counter()
        while queue or live or rerun:
            now = time.perf_counter() - t0
            while rerun and retry:
                req = rerun[0]
                slot = pool.admit(**job(req), host_checked=True)
                if slot is None:
                    if not live:
                        req.error = "does not fit the pool's budget"
                        req.finished = time.perf_counter() - t0
                        rerun.pop(0)
                        continue
                    retry = False
                    break
                live[slot] = req
                rerun.pop(0)
            while queue and retry and not rerun and (not realtime or queue[0].arrival <= now):
                req = queue[0]
                if head is None:
                    head = job(req)
                slot = pool.admit(**head)
                if slot is None:
                    if not live:
                        req.error = "does not fit the pool's budget"
                        queue.pop(0)
                        head = None
                        continue
                    retry = False
                    break
                req.admitted = time.perf_counter() - t0
                live[slot] = req
                queue.pop(0)
                head = None
            if not live and not rerun:
                if queue and realtime:
                    time.sleep(max(0.0, queue[0].arrival - (time.perf_counter() - t0)))
                continue
            pool.tick()
            for slot in [q for q in live if pool.poll(q)]:
                req = live.pop(slot)
                r = pool.result(slot)
                retry = True
                if r["status"] == L.SIM_WNOCONV and not getattr(req, "retried", 0):
                    req.retried = 1
                    rerun.append(req)
                    continue
                req.finished = time.perf_counter() - t0
                req.result = r
                if r["status"] != 0:
                    req.error = f"status {r['status']}: {r['worst']}"
                if on_done:
                    on_done(req)
        wall = time.perf_counter() - t0
    finally:
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
            "rerun_host_checked": sum(1 for r in ok if getattr(r, "retried", 0)),
            "failed": sum(1 for r in requests if r.error) - len(rejected),
            "wall_s": wall, "cell_steps_per_s": cell_steps / wall if wall > 0 else 0.0,
            "step_ms_p50": p(steps, 50), "step_ms_p99": p(steps, 99),
            "request_s_p50": p(lat, 50), "request_s_p99": p(lat, 99)}
