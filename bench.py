"""Benchmark: forward + adjoint cell-steps/s of the differentiable rollout.

Workload (one bench step): the 128^3 closed box with a moving ellipsoid
(9 shape parameters, 6 controls per step, seeded), curl-noise initial velocity,
dt = dx/2, 64 steps forward with a checkpoint every 8 steps, then the octant
loss, and the full adjoint (segment recomputation + per-step adjoint kernels +
shape / control gradients through the pose dynamics).  Inputs are resident on
the GPU before timing starts.  value = 128^3 * 64 * K / (wall time of K bench
steps), for the mixed-precision form (FP16 multigrid preconditioner); the
plain FP32 form is timed beside it.  Per-step latencies (HIP events around each
sim_step / sim_step_adjoint) give p50 / p99.

Both precision forms are timed the same way: CG iterations replayed from a
captured graph, no profiling.  After each form's timed rollouts, one more
rollout (outside the timed region) times the dominant kernel, the finest-level
multigrid post-smoother k_mg_up, with HIP events recorded by its own dispatches
on the launch stream; the roofline object sets its algorithmic bytes against
the MI355X HBM peak.  cg_iters gives the mean / max CG iterations per forward
and adjoint solve of the timed rollouts.

The cpu_baseline object times the FP64 oracle (child processes, before this
process touches the GPU) on a bounded sample: the same scene at 64^3, one
step forward + adjoint, once on one thread and once with every core allowed.
oracle_error compares the GPU's rollout of that sample (both precision forms,
benchmark tolerance) with the oracle's: final velocity, loss, shape and
control gradients.

Nested legs (objects in the same line, each skippable): "channel" (the
256x256x512 inflow / outflow channel with the B-spline wall, 200 steps
forward + adjoint), "serving" (a seeded request stream through the
continuous-batching loop against the same requests run serially in FP32),
"solids" (a 128^3 static union of four parametric solids, forward + adjoint
with the solids' parameter gradient) and "karman" (flow past a cylinder on
the x-independent slab at 512 x 1024 in the plane, forward steps).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 128
T = 64
EVERY = 8
# CG tolerance (relative residual) of every solve in the benchmark rollouts
CG_TOL = 1e-6
HBM_PEAK_GBS = 8000.0
ROOFLINE_KERNEL = "mg_up"
# A launch enqueued after the solver converged exits at once (about 1 us); the
# roofline averages launches of at least this length.
NOOP_MS = 0.003
# HBM bytes per (working) launch of the finest-level k_mg_up, FP16 form, from
# two rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch) scaled by the same counters of a plain 256 MiB device copy
# (--copy-probe 256: FETCH_SIZE reads 0.5x the bytes copied, WRITE_SIZE 1.0x);
# see profiles/mg_up_128_fp16_traffic.md.  Valid only for the kernel sources
# it was measured on (first 16 hex digits of their SHA-256).
TRAFFIC = {"fp16": 99928693}
TRAFFIC_SOURCES = {"paper_2405_14903_amd/csrc/nf_solver.hip": "3f9515635b656dad",
                   "paper_2405_14903_amd/csrc/nf_internal.h": "c1adffa6f7221945",
                   "paper_2405_14903_amd/csrc/nf_tile.h": "e8ea510b23a106e7"}


def measured_traffic(precision):
    import hashlib
    for rel, want in TRAFFIC_SOURCES.items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest()[:16] != want:
                    return None
        except OSError:
            return None
    return TRAFFIC.get(precision)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16", choices=["fp16", "bf16", "fp32"])
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison run")
    ap.add_argument("--solve-mode", default="host", choices=["host", "device"],
                    help="device: fixed iteration budget per solve, nothing waits on the host")
    ap.add_argument("--solve-budget", type=int, default=0, help="device solve mode's budget (0: from the warm-up)")
    ap.add_argument("--cold-start", action="store_true",
                    help="start every solve of the rollouts from zero (default: each adjoint solve starts from "
                         "the previous adjoint pressure)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-steps", type=int, default=1, help="steps of the oracle's sample rollout")
    ap.add_argument("--cpu-n", type=int, default=64, help="grid of the oracle's sample rollout")
    ap.add_argument("--cpu-oracle-run", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--summarize-trace", default=None, metavar="CSV",
                    help="only summarize a rocprofv3 kernel-trace CSV (kernel_trace.csv) as a markdown table")
    ap.add_argument("--summarize-title", default="kernel profile")
    ap.add_argument("--summarize-counters", default=None, metavar="CSV[,CSV]",
                    help="only summarize rocprofv3 --pmc counter CSVs (one per counter) of one kernel")
    ap.add_argument("--summarize-copy", default="", metavar="CSV[,CSV]",
                    help="with --summarize-counters: the same counters' CSVs of a --copy-probe run")
    ap.add_argument("--summarize-kernel", default="k_mg_up")
    ap.add_argument("--summarize-copy-mib", type=int, default=256)
    ap.add_argument("--summarize-grid", type=int, default=0,
                    help="with --summarize-trace: also report the working launches (>= 3 us) of the finest-level "
                         "k_mg_up, recognised by this grid size in threads")
    ap.add_argument("--workload", default="rollout128", choices=["rollout128", "channel", "serving"],
                    help="channel: the 256x256x512 inflow / outflow channel with the B-spline wall, "
                         "200 steps forward + adjoint, sqrt(T) checkpoints, total outflow flux loss, "
                         "gradients w.r.t. the 512 control amplitudes (FP16 V-cycle)")
    ap.add_argument("--channel-steps", type=int, default=200)
    ap.add_argument("--serve-requests", type=int, default=400, help="requests per rate (--workload serving)")
    ap.add_argument("--serve-rates", default="10,20,50,100,150,200", help="arrival rates (--workload serving)")
    ap.add_argument("--no-channel", action="store_true", help="skip the nested channel leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the nested serving leg")
    ap.add_argument("--no-solids", action="store_true", help="skip the nested parametric-solid leg")
    ap.add_argument("--no-karman", action="store_true", help="skip the nested Karman slab leg")
    ap.add_argument("--nested-solids-steps", type=int, default=32)
    ap.add_argument("--nested-karman-steps", type=int, default=50)
    ap.add_argument("--nested-channel-steps", type=int, default=200)
    ap.add_argument("--nested-serve-requests", type=int, default=48)
    ap.add_argument("--nested-serve-rate", type=float, default=100.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 launches): the reference kernel that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiling run")
    return ap.parse_args()


def copy_probe(mib, torch):
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "launches": 3}), flush=True)


class StepTimer:
    """HIP event pairs on torch's current stream (the stream the library uses)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {"fwd": [], "adj": [], "replay": []}
        self.open = None

    def begin(self, kind):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.open = (kind, e)

    def end(self, kind):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs[kind].append((self.open[1], e))

    def latencies(self, kind):
        return [a.elapsed_time(b) for a, b in self.pairs[kind]]


def run_form(precision, steps, warmup, scene, torch, roofline_pass=True, solve_mode="host", budget=0, warm=True):
    """Time `steps` rollouts of one precision form (graph-replayed CG, no
    profiling), then, outside the timed region, one more rollout with the
    finest-level k_mg_up timed by HIP events (the roofline kernel).

    solve_mode "device": after the warm-up (host-checked solves), every solve
    runs at most `budget` iterations (0: the warm-up's most iterations plus
    two, in whole check intervals of 8) with nothing waiting on the host; the
    solver reports are written on the device during the timed rollouts and
    read after them, and every solve must have converged."""
    from paper_2405_14903_amd.sim import Config, Sim
    from paper_2405_14903_amd.rollout import Rollout
    cfg = Config(n=scene.n, dx=scene.dx, dt=scene.dt, geom="ellipsoid", tol=CG_TOL, precision=precision,
                 max_iter=200)
    sim = Sim(cfg)
    u0 = torch.tensor(scene.u0, dtype=torch.float32, device="cuda")
    J = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(u0)
    iters = {"fwd": [], "adj": []}
    device_stats = []

    def one(timer):
        ro = Rollout.ellipsoid(sim, scene.theta0, scene.ctrl, every=EVERY, timer=timer,
                               warm_start="adjoint" if warm else False)
        if solve_mode == "device" and timer is not None:
            ro.device_stats = device_stats
        uT = ro.forward(u0)
        sim.loss_box(uT, J=J, g=g)
        ro.backward(g)
        ro.geometry_gradients()
        return ro

    most = 0
    for _ in range(warmup):
        ro = one(None)
        most = max([most] + ro.iters["fwd"] + ro.iters["adj"])
    if solve_mode == "device":
        budget = budget if budget > 0 else 8 * math.ceil((most + 2) / 8)
        sim.set_solve_mode("device", budget)
    print(f"[bench] {precision}: warmup done ({solve_mode} solves"
          f"{f', budget {budget}' if solve_mode == 'device' else ''})", file=sys.stderr, flush=True)
    timer = StepTimer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ro = one(timer)
        for k in iters:
            iters[k] += ro.iters[k]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    unconverged = 0
    for kind, st in device_stats:
        rep = st.as_dict()
        iters[kind].append(rep["iters"])
        unconverged += 0 if rep["converged"] else 1
    if solve_mode == "device":
        sim.set_solve_mode("host")
    print(f"[bench] {precision}: {steps} rollouts in {wall:.2f} s", file=sys.stderr, flush=True)
    prof = None
    if roofline_pass:
        sim.profile(ROOFLINE_KERNEL)
        one(None)
        torch.cuda.synchronize()
        prof = sim.profile_read(min_ms=NOOP_MS)
        sim.profile(None)
        print(f"[bench] {precision}: roofline pass done", file=sys.stderr, flush=True)
    fwd = timer.latencies("fwd")
    adj = timer.latencies("adj")
    rep = timer.latencies("replay")
    out = {
        "wall_s": wall,
        "cell_steps_per_s": (N ** 3) * T * steps / wall,
        "ms_per_rollout": 1e3 * wall / steps,
        "fwd_ms_p50": pct(fwd, 50), "fwd_ms_p99": pct(fwd, 99),
        "adj_ms_p50": pct(adj, 50), "adj_ms_p99": pct(adj, 99),
        "step_ms_p50": pct(fwd + adj, 50), "step_ms_p99": pct(fwd + adj, 99),
        "replay_ms_p50": pct(rep, 50), "replay_ms_p99": pct(rep, 99),
        "cg_iters": iter_summary(iters),
        "loss": float(J.item()),
        "solve_mode": solve_mode,
        "solve_start": "adjoint solves warm-started" if warm else "zero",
    }
    if solve_mode == "device":
        out["solve_budget"] = budget
        out["unconverged_solves"] = unconverged
    sim.close()
    return out, prof


def iter_summary(iters):
    """Mean / max CG iterations per forward solve (the timed forward and the
    recomputed segments) and per adjoint solve."""
    out = {}
    for k, v in iters.items():
        if v:
            out[k] = {"mean": round(sum(v) / len(v), 2), "max": max(v), "solves": len(v)}
    return out


def pct(v, q):
    if not v:
        return None
    s = sorted(v)
    i = min(len(s) - 1, max(0, int(math.ceil(q / 100.0 * len(s))) - 1))
    return round(s[i], 4)


def roofline(prof, precision, n3=(N, N, N), traffic=True):
    """Algorithmic bytes per launch of the finest-level up kernel of the
    V-cycle (coarse correction z' = z2 + 8 e(parent), two damped-Jacobi sweeps,
    r.z partials): it reads z2 (FP32), the coarse correction e (storage type,
    C/8 values), r (FP32), 1/diag (FP32 in every precision), the three
    face-fraction arrays (storage type; each face once) and the previous z
    (FP32, for the flexible direction coefficient), and writes z (FP32)."""
    es = 4 if precision == "fp32" else 2
    nx, ny, nz = n3
    C = nx * ny * nz
    F = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    bytes_per_launch = C * 4 + (C // 8) * es + C * 4 + C * 4 + F * es + C * 4 + C * 4
    ms, cnt = prof
    if not cnt:
        return None
    avg_s = ms / cnt / 1e3
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(precision) if traffic else None,
            "kernel": "k_mg_up (finest level, " + precision + ")", "launches": cnt,
            "avg_us": round(avg_s * 1e6, 2), "bytes_per_launch": bytes_per_launch}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_run(path, n, steps):
    """Child process: the FP64 oracle as it stands on the benchmark scene at
    n^3, `steps` steps forward + the full adjoint (octant loss); writes its
    results to `path` (npz) and prints its timing as one JSON line."""
    import numpy as np
    import scenes
    from oracle.mac import Grid
    from oracle.step import StepParams
    from oracle.rollout import EllipsoidRollout, octant_loss
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=n, steps=steps)
    g = Grid(sc.n, sc.dx)
    prm = StepParams(g, sc.dt, tol=1e-10)
    t0, c0 = time.perf_counter(), time.process_time()
    ro = EllipsoidRollout(prm, sc.u0, sc.theta0, sc.ctrl)
    uT = ro.forward()
    J, gT = octant_loss(g, uT)
    _, gth, gct = ro.backward(gT)
    wall, cpu = time.perf_counter() - t0, time.process_time() - c0
    np.savez(path, uT=uT, gth=gth, gct=gct, J=J)
    print(json.dumps({"wall_s": wall, "cpu_s": cpu}), flush=True)


def cpu_baseline(n, steps):
    """The oracle timed in child processes on the host cores, once limited to
    one thread and once allowed every core of this process' affinity mask
    (numpy / scipy's own threading: the sparse products it spends its time in
    run on one thread either way).  Returns (baseline object, path of the
    all-cores run's results)."""
    import subprocess
    import tempfile
    ncores = len(os.sched_getaffinity(0))
    runs = {}
    path = None
    for threads in (1, ncores):
        fd, out = tempfile.mkstemp(suffix=".npz")
        os.close(fd)
        env = dict(os.environ)
        for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[var] = str(threads)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-run", out, "--cpu-n", str(n),
                            "--cpu-steps", str(steps)], env=env, capture_output=True, text=True, check=True)
        runs[threads] = json.loads(r.stdout.strip().splitlines()[-1])
        print(f"[bench] oracle on {threads} thread(s): {runs[threads]['wall_s']:.1f} s", file=sys.stderr, flush=True)
        if threads == ncores:
            path = out
        else:
            os.remove(out)
    full, one = runs[ncores], runs[1]
    rate = lambda r: round(n ** 3 * steps / r["wall_s"], 1)  # noqa: E731
    cores = max(1, round(full["cpu_s"] / full["wall_s"]))
    base = {"value": rate(full), "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"the benchmark scene (moving ellipsoid, curl noise, same shape parameters and controls) at "
                      f"{n}^3, {steps} step(s) forward + adjoint with the octant loss (FP64 numpy / scipy, "
                      f"Jacobi-PCG to 1e-10), {full['wall_s']:.1f} s wall, {full['cpu_s']:.1f} s CPU with "
                      f"{ncores} threads allowed on {cpu_model()}; cores = CPU time / wall time",
            "threads_allowed": ncores,
            "single_thread": {"value": rate(one), "wall_s": round(one["wall_s"], 2)}}
    return base, path


def oracle_check(path, n, steps, torch):
    """Error against the FP64 oracle on the same scene at n^3 and `steps`
    steps: the GPU rollout as the benchmark runs it (benchmark tolerance,
    warm-started adjoint solves) in both precision forms, final velocity and
    shape / control gradients."""
    import numpy as np
    import scenes
    from paper_2405_14903_amd.sim import Config, Sim
    from paper_2405_14903_amd.rollout import Rollout
    ref = np.load(path)
    sc = scenes.scene_ellipsoid_rollout(seed=0, n=n, steps=steps)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
    out = {"grid": [n, n, n], "steps": steps, "cg_tol": CG_TOL}
    for prec in ("fp16", "fp32"):
        cfg = Config(n=sc.n, dx=sc.dx, dt=sc.dt, geom="ellipsoid", tol=CG_TOL, precision=prec, max_iter=200)
        with Sim(cfg) as sim:
            u0 = torch.tensor(sc.u0, dtype=torch.float32, device="cuda")
            ro = Rollout.ellipsoid(sim, sc.theta0, sc.ctrl, every=EVERY, warm_start="adjoint")
            uT = ro.forward(u0)
            J, g = sim.loss_box(uT)
            ro.backward(g)
            gth, gct = ro.geometry_gradients()
            torch.cuda.synchronize()
            uh = uT.double().cpu().numpy()
        out[prec] = {"velocity_rel_l2": rel(uh, ref["uT"]), "loss_rel": abs(float(J.item()) - float(ref["J"])) /
                     abs(float(ref["J"])), "theta_grad_rel_l2": rel(gth, ref["gth"]),
                     "ctrl_grad_rel_l2": rel(gct, ref["gct"])}
    os.remove(path)
    return out


def channel_leg(args, torch, steps, precision, profile=True):
    """The channel configuration: a short warm-up rollout, then one timed
    rollout of `steps` steps forward + adjoint.  Returns its summary."""
    import scenes
    from paper_2405_14903_amd.sim import Config, Sim
    from paper_2405_14903_amd.rollout import Rollout
    n3, T = scenes.CHANNEL_FULL_N, steps
    sc = scenes.scene_channel(seed=0, n=n3, steps=T)
    kn, f, amp = sc.extra["knots"], sc.extra["f"], sc.extra["amp"]
    cfg = Config(n=n3, dx=sc.dx, dt=sc.dt, bc=("wall", "wall", "wall", "wall", "inflow", "outflow"),
                 inflow_speed=1.0, geom="wall", tol=CG_TOL, precision=precision, max_iter=400)
    sim = Sim(cfg)
    u0 = torch.tensor(sc.u0, dtype=torch.float32, device="cuda")
    zero = torch.zeros_like(u0)

    def one(steps, timer):
        ro = Rollout.channel(sim, kn, f, amp, steps, every="sqrt", timer=timer)
        ro.forward(u0)
        ro.backward(zero)
        return ro

    one(4, None)
    torch.cuda.synchronize()
    print("[bench] channel: warmup done", file=sys.stderr, flush=True)
    timer = StepTimer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ro = one(T, timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] channel: {T} steps forward + adjoint in {wall:.2f} s", file=sys.stderr, flush=True)
    prof = None
    if profile:
        sim.profile(ROOFLINE_KERNEL)
        one(min(T, 16), None)
        torch.cuda.synchronize()
        prof = sim.profile_read(min_ms=NOOP_MS)
        sim.profile(None)
    gk = ro.g_steps.sum(dim=0)
    fwd, adj = timer.latencies("fwd"), timer.latencies("adj")
    C = n3[0] * n3[1] * n3[2]
    out = {
        "value": round(C * T / wall, 1), "unit": "cell-steps/s", "wall_s": round(wall, 3),
        "workload": f"256x256x512 channel, B-spline wall (16x32 control amplitudes), inflow / outflow, "
                    f"{T} steps forward + adjoint, sqrt(T) checkpoints (every {ro.K}), total outflow flux",
        "precision": precision, "cg_tol": CG_TOL,
        "latency_ms": {"step_p50": pct(fwd + adj, 50), "step_p99": pct(fwd + adj, 99),
                       "fwd_p50": pct(fwd, 50), "fwd_p99": pct(fwd, 99), "adj_p50": pct(adj, 50),
                       "adj_p99": pct(adj, 99)},
        "cg_iters": iter_summary(ro.iters),
        "loss": float(ro.J.item()), "knot_gradient_norm": float(gk.norm()),
        "roofline": roofline(prof, precision, n3, traffic=False) if prof else None,
    }
    sim.close()
    return out


def family_us(sim, family, run, torch):
    """Average HIP-event time (us) of one kernel family's working launches
    while `run()` executes."""
    sim.profile(family)
    run()
    torch.cuda.synchronize()
    ms, cnt = sim.profile_read(min_ms=NOOP_MS)
    sim.profile(None)
    return round(1e3 * ms / cnt, 2) if cnt else None


def solids_leg(torch, steps, precision):
    """The parametric-solid geometry: a static CSG union of four polar-Bezier
    solids in the 128^3 closed box, `steps` steps forward + adjoint with the
    octant loss and dJ/dtheta of all 4 x 44 solid parameters."""
    import scenes
    from paper_2405_14903_amd.sim import Config, Sim
    from paper_2405_14903_amd.rollout import Rollout
    n = N
    sc = scenes.scene_solids(seed=0, n=n, count=4)
    th = sc.extra["theta"]
    cfg = Config(n=sc.n, dx=sc.dx, dt=sc.dt, geom="bezier", n_solids=4, tol=CG_TOL, precision=precision,
                 max_iter=200)
    sim = Sim(cfg)
    u0 = torch.tensor(sc.u0, dtype=torch.float32, device="cuda")

    def one(T, timer):
        ro = Rollout(sim, T, lambda k: (th, None), every=EVERY, grad_geometry=True, timer=timer)
        J, g = sim.loss_box(ro.forward(u0))
        ro.backward(g)
        return ro, J

    one(4, None)
    torch.cuda.synchronize()
    timer = StepTimer(torch)
    t0 = time.perf_counter()
    ro, J = one(steps, timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gth = ro.g_steps.sum(dim=0)
    phi_us = family_us(sim, "geom_phi", lambda: one(2, None), torch)
    adj_us = family_us(sim, "adj_faces", lambda: one(2, None), torch)
    fwd, adj = timer.latencies("fwd"), timer.latencies("adj")
    print(f"[bench] solids: {steps} steps forward + adjoint in {wall:.2f} s", file=sys.stderr, flush=True)
    out = {
        "value": round(n ** 3 * steps / wall, 1), "unit": "cell-steps/s", "wall_s": round(wall, 3),
        "workload": f"{n}^3 closed box, static union of 4 parametric solids (polar Bezier cross-sections, "
                    f"3 key sections, 4 x 44 parameters), {steps} steps forward + adjoint, checkpoint every "
                    f"{EVERY}, octant loss, dJ/dtheta",
        "precision": precision, "cg_tol": CG_TOL,
        "latency_ms": {"fwd_p50": pct(fwd, 50), "fwd_p99": pct(fwd, 99), "adj_p50": pct(adj, 50),
                       "adj_p99": pct(adj, 99)},
        "cg_iters": iter_summary(ro.iters),
        "geometry_us": {"phi_solids": phi_us, "adjoint_faces_and_solids": adj_us},
        "loss": float(J.item()), "theta_gradient_norm": float(gth.norm()),
    }
    sim.close()
    return out


def karman_leg(torch, steps, precision, n=(32, 512, 1024)):
    """Flow past a cylinder on the x-independent slab at the paper's 512 x 1024
    resolution in the plane (32 cells thick, the least that coarsens to the
    multigrid bottom): `steps` forward steps at Re = 100, timed."""
    import scenes
    from paper_2405_14903_amd.sim import Config, Sim
    sc = scenes.scene_karman(n=n, diameter=0.1, dt=1e-3)
    th = sc.extra["theta"]
    cfg = Config(n=sc.n, dx=sc.dx, dt=sc.dt, nu=1e-3, bc=sc.extra["bc"], inflow_speed=sc.extra["inflow"],
                 geom="bezier", n_solids=1, tol=CG_TOL, precision=precision, max_iter=400)
    sim = Sim(cfg)
    a = torch.tensor(sc.u0, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    iters = []
    for _ in range(3):
        b, st = sim.step(a, th, u_out=b)
        a, b = b, a
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b, st = sim.step(a, th, u_out=b)
        iters.append(st["iters"])
        a, b = b, a
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    C = n[0] * n[1] * n[2]
    print(f"[bench] karman: {steps} steps in {wall:.2f} s", file=sys.stderr, flush=True)
    sim.close()
    return {"value": round(C * steps / wall, 1), "unit": "cell-steps/s", "wall_s": round(wall, 3),
            "ms_per_step": round(1e3 * wall / steps, 3),
            "workload": f"flow past a cylinder (diameter 0.1, Re 100, nu 1e-3, inflow 1), x-independent slab "
                        f"{n[0]} x {n[1]} x {n[2]} ({n[1]} x {n[2]} in the plane), dt 1e-3, {steps} forward "
                        f"steps after 3 warm-up steps",
            "precision": precision, "cg_tol": CG_TOL, "cg_iters": iter_summary({"fwd": iters})}


def run_channel(args, torch):
    """--workload channel: the channel leg as the one JSON line."""
    leg = channel_leg(args, torch, args.channel_steps, args.precision)
    rec = {
        "metric": "fwd+adjoint cell-steps/s, 256x256x512 channel (mixed); p50/p99 step latency",
        "value": leg["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1e3 * leg["wall_s"], 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype_of(args.precision), "data": "synthetic",
        "config": {"workload": leg["workload"], "grid": [256, 256, 512], "precision": args.precision,
                   "cg_tol": CG_TOL},
        "latency_ms": leg["latency_ms"], "cg_iters": leg["cg_iters"], "loss": leg["loss"],
        "knot_gradient_norm": leg["knot_gradient_norm"], "roofline": leg["roofline"], "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def dtype_of(precision):
    return "f32+f16" if precision == "fp16" else ("f32+bf16" if precision == "bf16" else "f32")


def serving_leg(torch, n_req, rates, precision, seed=0):
    """The serving configuration on a bounded stream: `n_req` seeded requests
    per arrival rate (Poisson arrivals; grids {32, 48, 64, 96, 128, 192}^3,
    8 to 64 steps; one in ten a pressure projection, the rest half
    forward-only and half forward + adjoint), served with continuous batching
    and the mixed-precision form within an HBM budget, against the same
    requests run one at a time in plain FP32 on the same arrival schedule."""
    from paper_2405_14903_amd.serving import make_stream, serve, serve_pool, serve_serial
    budget = 200 << 30
    sizes = (32, 48, 64, 96, 128, 192)
    out = {"workload": f"{n_req} requests per rate, Poisson arrivals, grids {{32..192}}^3, 8-64 steps, 10% pressure "
                       f"projections, the rest half forward-only and half forward + adjoint; continuous batching "
                       f"(8 episodes, {budget >> 30} GiB budget) with the {precision} V-cycle and device-mode "
                       f"solves, by the Python scheduler (served) and by the library's native pool (native_pool), "
                       f"against serial plain FP32 on the same schedule",
           "rates": {}}
    for rate in rates:
        served = serve(make_stream(n_req, rate, seed=seed), budget_bytes=budget, precision=precision, max_active=8,
                       realtime=True, warm_sizes=sizes)
        native = serve_pool(make_stream(n_req, rate, seed=seed), budget_bytes=budget, precision=precision,
                            max_active=8, realtime=True, warm_sizes=sizes)
        serial = serve_serial(make_stream(n_req, rate, seed=seed), precision="fp32", warm_sizes=sizes)
        print(f"[bench] serving at {rate:g} req/s: served {served['cell_steps_per_s'] / 1e6:.1f} M, native pool "
              f"{native['cell_steps_per_s'] / 1e6:.1f} M, serial {serial['cell_steps_per_s'] / 1e6:.1f} M "
              f"cell-steps/s", file=sys.stderr, flush=True)
        keep = ("completed", "failed", "rejected", "rerun_host_checked", "wall_s", "cell_steps_per_s", "step_ms_p50", "step_ms_p99",
                "request_s_p50", "request_s_p99")
        out["rates"][f"{rate:g}"] = {
            "served": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in served.items() if k in keep},
            "native_pool": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in native.items()
                            if k in keep and not k.startswith("step_ms")},
            "serial_fp32": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in serial.items() if k in keep},
            "throughput_over_serial": round(served["cell_steps_per_s"] / serial["cell_steps_per_s"], 3)
            if serial["cell_steps_per_s"] else None,
            "native_pool_over_serial": round(native["cell_steps_per_s"] / serial["cell_steps_per_s"], 3)
            if serial["cell_steps_per_s"] else None,
            "step_p99_over_serial": round(served["step_ms_p99"] / serial["step_ms_p99"], 3)
            if served["step_ms_p99"] and serial["step_ms_p99"] else None}
    return out


def run_serving(args, torch):
    """--workload serving: the serving leg as the one JSON line."""
    rates = [float(r) for r in args.serve_rates.split(",")]
    leg = serving_leg(torch, args.serve_requests, rates, args.precision)
    first = leg["rates"][f"{rates[0]:g}"]
    # the headline is the library's own serving pool (sim_pool_*); the Python
    # scheduler and serial FP32 are reported beside it
    rec = {
        "metric": "serving: cell-steps/s of the native pool (Python scheduler and serial FP32 beside it)",
        "value": round(first["native_pool"]["cell_steps_per_s"], 1), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * first["native_pool"]["wall_s"], 3),
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_of(args.precision), "data": "synthetic",
        "config": {"workload": leg["workload"], "rates": rates, "precision": args.precision},
        "serving": leg, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def summarize_trace(path, title, fine_grid=0):
    """Markdown summary of a rocprofv3 --kernel-trace CSV: one row per kernel
    name and grid size (the grid tells the multigrid levels apart)."""
    import csv
    rows = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r.get("Kernel_Name", "?")
            name = name.split("(")[0].replace("void ", "").replace("nf::", "").replace("TileShape", "T")
            grid = int(r.get("Grid_Size_X", r.get("Grid_Size", "0")) or 0) * int(r.get("Grid_Size_Y", "1") or 1) * \
                int(r.get("Grid_Size_Z", "1") or 1)
            wg = int(r.get("Workgroup_Size_X", r.get("Workgroup_Size", "0")) or 0) * \
                int(r.get("Workgroup_Size_Y", "1") or 1) * int(r.get("Workgroup_Size_Z", "1") or 1)
            us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            rows.setdefault((name, grid, wg), []).append(us)
    total = sum(sum(v) for v in rows.values())
    ndisp = sum(len(v) for v in rows.values())
    print(f"# {title}\n")
    print(f"Source: `{os.path.basename(path)}` (rocprofv3 kernel trace).  Grid = launch size in threads.\n")
    if fine_grid:
        up = [u for (name, grid, wg), v in rows.items() if "k_mg_up" in name and grid == fine_grid for u in v]
        work = [u for u in up if u >= NOOP_MS * 1e3]
        avg = sum(work) / len(work) if work else 0.0
        print(f"Finest-level `k_mg_up` (grid {fine_grid}): {len(up)} launches; the {len(work)} of at least "
              f"{NOOP_MS * 1e3:g} us (the others were enqueued after a solve converged and exit at once) average "
              f"{avg:.2f} us.\n")
    print("| kernel | grid (threads) | wg | calls | avg us | min us | max us | total ms | % of kernel time |")
    print("|---|---|---|---|---|---|---|---|---|")
    for (name, grid, wg), v in sorted(rows.items(), key=lambda kv: -sum(kv[1]))[:40]:
        print(f"| `{name}` | {grid} | {wg} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
              f"{sum(v) / 1e3:.2f} | {100 * sum(v) / total:.1f} |")
    print(f"\nTotal kernel time {total / 1e3:.1f} ms over {ndisp} dispatches.")


def summarize_counters(paths, copy_paths, kernel, grid, copy_mib):
    """Markdown summary of rocprofv3 --pmc runs: per counter (FETCH_SIZE,
    WRITE_SIZE; KiB per dispatch) the mean over the working dispatches of one
    kernel (name containing `kernel`, launch grid `grid` threads; a working
    dispatch reads more than a quarter of the largest one, the others were
    enqueued after a solve converged and exit at once), scaled by the same
    counter's reading for a plain device copy of copy_mib MiB."""
    import csv

    def rows(path):
        with open(path, newline="") as f:
            return list(csv.DictReader(f))
    total = 0.0
    print(f"| counter | copy KiB per dispatch | scale | working dispatches | KiB per working dispatch | bytes |")
    print("|---|---|---|---|---|---|")
    for path, cpath in zip(paths, copy_paths):
        rs = [r for r in rows(path) if kernel in r["Kernel_Name"] and int(r.get("Grid_Size", 0) or 0) == grid]
        name = rs[0]["Counter_Name"] if rs else "?"
        vals = [float(r["Counter_Value"]) for r in rs]
        cs = [float(r["Counter_Value"]) for r in rows(cpath) if "copy" in r["Kernel_Name"].lower()]
        cmean = sum(cs) / len(cs) if cs else float("nan")
        scale = copy_mib * 1024.0 / cmean if cs else float("nan")
        top = max(vals) if vals else 0.0
        work = [v for v in vals if v > 0.25 * top]
        mean = sum(work) / len(work) if work else 0.0
        b = mean * 1024.0 * scale
        total += b
        print(f"| {name} | {cmean:.1f} | x {scale:.4f} | {len(work)} of {len(vals)} | {mean:.1f} | {b / 1e6:.2f} MB |")
    print(f"\nTotal HBM traffic per working dispatch: **{total / 1e6:.2f} MB** ({int(round(total))} bytes).")


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters.split(","), args.summarize_copy.split(","), args.summarize_kernel,
                           args.summarize_grid, args.summarize_copy_mib)
        return
    if args.cpu_oracle_run:
        cpu_oracle_run(args.cpu_oracle_run, args.cpu_n, args.cpu_steps)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.summarize_title, args.summarize_grid)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the rollout of one episode is a "
              f"single-GPU workload here, and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)
    # the oracle's CPU leg runs first, in child processes, before this process
    # touches the GPU
    cpu, oracle_path = (None, None)
    if not args.no_cpu and args.workload == "rollout128" and not args.copy_probe:
        cpu, oracle_path = cpu_baseline(args.cpu_n, args.cpu_steps)
    import torch
    import scenes
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe, torch)
        return
    if args.workload == "channel":
        run_channel(args, torch)
        return
    if args.workload == "serving":
        run_serving(args, torch)
        return
    scene = scenes.scene_ellipsoid_rollout(seed=0, n=N, steps=T)
    main_form, prof = run_form(args.precision, args.steps, args.warmup, scene, torch, solve_mode=args.solve_mode,
                               budget=args.solve_budget, warm=not args.cold_start)
    cmp_form = None
    if not args.no_compare and args.precision != "fp32":
        cmp_form, cmp_prof = run_form("fp32", args.steps, args.warmup, scene, torch, solve_mode=args.solve_mode,
                                      budget=args.solve_budget, warm=not args.cold_start)
    rec = {
        "metric": "fwd+adjoint cell-steps/s at 128^3 (mixed vs FP32); p50/p99 step latency",
        "value": round(main_form["cell_steps_per_s"], 1),
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_form["ms_per_rollout"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_of(args.precision),
        "data": "synthetic",
        "config": {"workload": "128^3 closed box, moving ellipsoid (9 shape params, 6 controls/step), "
                               "64 steps forward + adjoint, checkpoint every 8, octant loss",
                   "grid": [N, N, N], "steps_per_rollout": T, "checkpoint_every": EVERY,
                   "precision": args.precision, "cg_tol": CG_TOL,
                   "recompute": "segments replayed from the pressures kept by the first forward (no solve)"},
        "latency_ms": {"step_p50": main_form["step_ms_p50"], "step_p99": main_form["step_ms_p99"],
                       "fwd_p50": main_form["fwd_ms_p50"], "fwd_p99": main_form["fwd_ms_p99"],
                       "adj_p50": main_form["adj_ms_p50"], "adj_p99": main_form["adj_ms_p99"],
                       "replay_p50": main_form["replay_ms_p50"], "replay_p99": main_form["replay_ms_p99"]},
        "cg_iters": main_form["cg_iters"],
        "solve": {k: main_form[k] for k in ("solve_mode", "solve_start", "solve_budget", "unconverged_solves")
                  if k in main_form},
        "roofline": roofline(prof, args.precision),
    }
    if cmp_form:
        rec["fp32"] = {"value": round(cmp_form["cell_steps_per_s"], 1),
                       "ms_per_step": round(cmp_form["ms_per_rollout"], 3),
                       "step_p50_ms": cmp_form["step_ms_p50"], "step_p99_ms": cmp_form["step_ms_p99"],
                       "cg_iters": cmp_form["cg_iters"],
                       "solve": {k: cmp_form[k] for k in ("solve_mode", "solve_start", "solve_budget",
                                                          "unconverged_solves") if k in cmp_form},
                       "roofline": roofline(cmp_prof, "fp32", traffic=False)}
        rec["mixed_over_fp32"] = round(main_form["cell_steps_per_s"] / cmp_form["cell_steps_per_s"], 3)
    if oracle_path:
        rec["oracle_error"] = oracle_check(oracle_path, args.cpu_n, args.cpu_steps, torch)
    if not args.no_channel:
        rec["channel"] = channel_leg(args, torch, args.nested_channel_steps, args.precision, profile=False)
    if not args.no_serving:
        rec["serving"] = serving_leg(torch, args.nested_serve_requests, [args.nested_serve_rate], args.precision)
    if not args.no_solids:
        rec["solids"] = solids_leg(torch, args.nested_solids_steps, args.precision)
    if not args.no_karman:
        rec["karman"] = karman_leg(torch, args.nested_karman_steps, args.precision)
    rec["cpu_baseline"] = cpu
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
