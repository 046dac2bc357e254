"""Continuous batching of droplet simulations on one GPU.

Jobs (2D oscillating droplets of uneven particle counts and parameters) arrive
as a Poisson process.  A job is admitted into a device pool as soon as the
pool's HBM budget holds it; every scheduler tick advances all admitted jobs in
the same launches (each job keeps its own time steps); finished jobs are read
out and released, freeing room for queued ones.

Jobs differ several-fold in acoustic substeps per advection step (Eqs. 16-18),
and a tick lasts as long as its longest job.  A tick therefore gives a job
that needs fewer substeps per step proportionally more advection steps (up to
max_steps_per_tick), so that all jobs fill the tick; max_steps_per_tick=1
steps every job once per tick.  The loop records each job's advection steps
with their latency, the tick's wall time shared out over the steps the job
took in it, and reports p50/p99 per-step latency (and per tick) beside the
aggregate particle-steps/s.  It also reports each job's step interval: the
wall time from its admission or previous tick to the end of its tick, shared
out over the steps it took, which includes the time the loop spends admitting
and releasing other jobs.  Job payloads are built before the clock starts, as
a request carries its particles when it arrives.

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


# health bits that fault a system (RSPH_HEALTH_*; 16 is an input check only)
FAULT_BITS = 1 | 2 | 4 | 8 | 32


def build_job(desc):
    return WL.oscillating_ellipse_2d(desc["n"], desc["aspect"], desc["ratio"], desc["gamma"],
                                     seed=desc["seed"])


def steps_this_tick(sps, left, cap):
    """Advection steps per job for one tick: the job with the most substeps
    per step takes one; a job needing fewer takes as many as fit in the same
    number of substeps (at most cap and its steps left).  A job whose count is
    not known yet takes one."""
    known = [v for v in sps if v > 0]
    ref = max(known) if known else 0
    out = []
    for v, l in zip(sps, left):
        n = 1 if (v <= 0 or ref == 0) else max(1, ref // v)
        out.append(int(max(1, min(n, cap, l))))
    return out


def serve(job_descs, steps_per_job=200, rate_hz=None, budget_bytes=4 << 30, precision=rsph.MIXED,
          log=None, keep_results=False, max_seconds=None, max_steps_per_tick=1, max_admits_per_tick=0,
          builder=build_job):
    """Runs the request loop to completion.  rate_hz: Poisson arrival rate
    (None: all jobs arrive at t = 0).  max_admits_per_tick > 0 bounds the
    admissions between two ticks (each one stalls the running jobs).  Returns a
    summary dictionary.  A job whose health check trips is released and reported
    (jobs_failed, failed_health) while the others go on.  builder(desc) makes a
    job's parameters and particles."""
    rng = np.random.Generator(np.random.PCG64(12345))
    n_jobs = len(job_descs)
    if rate_hz:
        arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_jobs))
    else:
        arrivals = np.zeros(n_jobs)
    built = {k: builder(d) for k, d in enumerate(job_descs)}
    pool = rsph.Pool(2, precision=precision, budget_bytes=budget_bytes)
    queue = collections.deque()
    active = {}  # job index -> [system, steps done, n particles, end of its last tick or admission]
    step_latency = []
    step_interval = []
    tick_latency = []
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
        admitted = 0
        while queue and (max_admits_per_tick <= 0 or admitted < max_admits_per_tick or not active):
            k = queue[0]
            w = built[k]
            try:
                s = pool.admit(w["params"], w["pos"], w["vel"], w["phase"])
            except rsph.RsphError as e:
                if e.name == "EBUSY" and active:
                    break
                raise
            queue.popleft()
            admitted += 1
            active[k] = [s, 0, w["pos"].shape[0], time.perf_counter()]
        queue_depth.append(len(queue))
        if not active:
            # idle until the next arrival
            if next_arrival < n_jobs:
                time.sleep(max(0.0, arrivals[next_arrival] - (time.perf_counter() - t0)))
            continue
        order = sorted(active)
        if max_steps_per_tick > 1:
            sps = [active[k][0].step_counts()["substeps_per_step"] for k in order]
            n_tick = steps_this_tick(sps, [steps_per_job - active[k][1] for k in order], max_steps_per_tick)
        else:
            n_tick = [1] * len(order)
        ta = time.perf_counter()
        failed_now = {}
        try:
            pool.step([active[k][0] for k in order], n_tick)
        except rsph.RsphError as e:
            # one job's health check tripped: the others took their steps;
            # the faulted ones are released and reported, the loop goes on
            if e.name != "ENUMERIC":
                raise
            for k in order:
                h = active[k][0].observables()["health"]
                if h & FAULT_BITS:
                    failed_now[k] = h
            if not failed_now:
                raise
        tb = time.perf_counter()
        dt = tb - ta
        tick_latency.append(dt)
        for k, h in failed_now.items():
            s = active[k][0]
            finished[k] = {"n": active[k][2], "done_at": time.perf_counter() - t0,
                           "arrived": float(arrivals[k]), "result": None, "failed": int(h),
                           "steps": active[k][1]}
            pool.release(s)
            built.pop(k, None)
            del active[k]
            if log:
                log(f"job {k} failed (health bits 0x{h:x}) after {finished[k]['steps']} steps; released")
        steps_of = dict(zip(order, n_tick))
        order = [k for k in order if k not in failed_now]
        n_tick = [steps_of[k] for k in order]
        for k, n in zip(order, n_tick):
            active[k][1] += n
            particle_steps += active[k][2] * n
            step_latency.extend([dt / n] * n)
            step_interval.extend([(tb - active[k][3]) / n] * n)
            active[k][3] = tb
        for k in order:
            s, done, n, _ = active[k]
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
    failed = {k: f["failed"] for k, f in finished.items() if f.get("failed")}
    lat = np.array(step_latency) if step_latency else np.zeros(1)
    tick = np.array(tick_latency) if tick_latency else np.zeros(1)
    gap = np.array(step_interval) if step_interval else np.zeros(1)
    summary = {
        "jobs": len(finished) - len(failed),
        "jobs_failed": len(failed),
        "failed_health": failed,
        "wall_s": wall,
        "particle_steps": particle_steps,
        "particle_steps_per_s": particle_steps / wall if wall > 0 else 0.0,
        "step_latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
        "step_latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
        "tick_latency_p50_ms": float(np.percentile(tick, 50) * 1e3),
        "tick_latency_p99_ms": float(np.percentile(tick, 99) * 1e3),
        "step_interval_p50_ms": float(np.percentile(gap, 50) * 1e3),
        "step_interval_p99_ms": float(np.percentile(gap, 99) * 1e3),
        "max_steps_per_tick": max_steps_per_tick,
        "max_queue_depth": int(max(queue_depth) if queue_depth else 0),
        "turnaround_p50_s": float(np.median([f["done_at"] - f["arrived"] for f in finished.values()
                                             if not f.get("failed")]))
        if len(finished) > len(failed) else math.nan,
    }
    if keep_results:
        summary["results"] = {k: f["result"] for k, f in finished.items() if not f.get("failed")}
    pool.close()
    return summary
