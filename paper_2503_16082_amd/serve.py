"""Continuous batching of droplet simulations on one GPU.

Jobs (2D oscillating droplets of uneven particle counts and parameters) arrive
as a Poisson process.  A job is admitted into a device pool as soon as the
pool's HBM budget holds it; every scheduler tick advances all admitted jobs by
one advection step in the same launches (each job keeps its own time steps);
finished jobs are read out and released, freeing room for queued ones.  The
loop records, per job, the wall time of each advection step it took part in,
and reports p50/p99 per-step latency beside the aggregate particle-steps/s.

Host-side scheduling only: all stepping runs in the HIP library through the
pool entry points of the C-ABI.
"""
from __future__ import annotations

import collections
import math
import time

import numpy as np

from . import rsph
from . import workloads as WL


def build_job(desc):
    return WL.oscillating_ellipse_2d(desc["n"], desc["aspect"], desc["ratio"], desc["gamma"],
                                     seed=desc["seed"])


def serve(job_descs, steps_per_job=200, rate_hz=None, budget_bytes=4 << 30, precision=rsph.MIXED,
          log=None, keep_results=False, max_seconds=None):
    """Runs the request loop to completion.  rate_hz: Poisson arrival rate
    (None: all jobs arrive at t = 0).  Returns a summary dictionary."""
    rng = np.random.Generator(np.random.PCG64(12345))
    n_jobs = len(job_descs)
    if rate_hz:
        arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_jobs))
    else:
        arrivals = np.zeros(n_jobs)
    built = {}
    pool = rsph.Pool(2, precision=precision, budget_bytes=budget_bytes)
    queue = collections.deque()
    active = {}  # job index -> [system, steps done, n particles]
    step_latency = []
    finished = {}
    next_arrival = 0
    particle_steps = 0
    queue_depth = []
    t0 = time.perf_counter()
    while len(finished) < n_jobs:
        now = time.perf_counter() - t0
        if max_seconds and now > max_seconds:
            break
        while next_arrival < n_jobs and arrivals[next_arrival] <= now:
            queue.append(next_arrival)
            next_arrival += 1
        # admission, first come first served, as long as the budget allows
        while queue:
            k = queue[0]
            if k not in built:
                built[k] = build_job(job_descs[k])
            w = built[k]
            try:
                s = pool.admit(w["params"], w["pos"], w["vel"], w["phase"])
            except rsph.RsphError as e:
                if e.name == "EBUSY" and active:
                    break
                raise
            queue.popleft()
            active[k] = [s, 0, w["pos"].shape[0]]
        queue_depth.append(len(queue))
        if not active:
            # idle until the next arrival
            if next_arrival < n_jobs:
                time.sleep(max(0.0, arrivals[next_arrival] - (time.perf_counter() - t0)))
            continue
        order = sorted(active)
        ta = time.perf_counter()
        pool.step([active[k][0] for k in order], [1] * len(order))
        dt = time.perf_counter() - ta
        for k in order:
            active[k][1] += 1
            particle_steps += active[k][2]
            step_latency.append(dt)
        for k in order:
            s, done, n = active[k]
            if done >= steps_per_job:
                res = None
                if keep_results:
                    res = {f: s.read(f) for f in ["pos", "vel", "rho"]}
                finished[k] = {"n": n, "done_at": time.perf_counter() - t0,
                               "arrived": float(arrivals[k]), "result": res}
                pool.release(s)
                built.pop(k, None)
                del active[k]
                if log:
                    log(f"job {k} done ({n} particles) at {finished[k]['done_at']:.2f}s, "
                        f"{len(active)} active, {len(queue)} queued")
    wall = time.perf_counter() - t0
    lat = np.array(step_latency) if step_latency else np.zeros(1)
    summary = {
        "jobs": len(finished),
        "wall_s": wall,
        "particle_steps": particle_steps,
        "particle_steps_per_s": particle_steps / wall if wall > 0 else 0.0,
        "step_latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "step_latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_queue_depth": int(max(queue_depth) if queue_depth else 0),
        "turnaround_p50_s": float(np.median([f["done_at"] - f["arrived"] for f in finished.values()]))
        if finished else math.nan,
    }
    if keep_results:
        summary["results"] = {k: f["result"] for k, f in finished.items()}
    pool.close()
    return summary
