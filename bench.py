"""Benchmark of the Riemann-SPH multiphase surface-tension hot path on one GPU.

A step is one advection step of the dual-criteria scheme: rebinning, neighbour
lists, density summation, viscous acceleration, correction matrix and position
shift, then every acoustic substep (colour gradient, Riemann pressure with the
surface stress and penalty force, kick, continuity) until the advection step is
covered.  The default workload is the largest single-GPU one: the 3D droplet
impact onto a liquid pool, 8,388,608 particles (drop D = 1 at 32 particles per
unit length, pool depth 2 in an 8 x 8 x 4 air-filled periodic box, density
ratio 1000, viscosity ratio 100, Re = 1e4, We = 2.5e4), in the mixed precision
form (FP32 pair loops, FP64 state), with the penalty force on.  Inputs are
synthetic and already resident in device memory when the timed region starts.

The same run also measures the FP64 form on the same steps, the single-step
acceleration error of the mixed and FP64 forms against the FP64 oracle on a
sample chosen from the inputs, the FP64 oracle itself on the host cores (one
advection step of the same workload), and the served form: a stream of 256 2D
droplet jobs admitted by HBM budget into one pool, with p50/p99 per-step
latency.

Prints ONE JSON line.  Everything else goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2503_16082_amd import rsph  # noqa: E402
from paper_2503_16082_amd import workloads as WL  # noqa: E402

# MI355X vector peaks for the ALU fraction.  The published FP32 figure
# (157.3 TFLOP/s) needs packed FP32 instructions, which this build does not
# generate (-packed-fp32-ops), so FP32 is priced at the non-packed rate:
# 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s, the FP64 rate.
PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
# working sets below this are served from the 256 MB Infinity Cache, where an
# HBM fraction is no evidence of HBM use
MALL_BYTES = 256 << 20
PEAK_HBM_GBS = 8000.0

# Algorithmic operations per neighbour pair of the force pass (Riemann pressure,
# Eqs. 7-12) and its surface part (stress divergence and projected penalty,
# Eqs. 24, 27, 30, 33, near-interface pairs only), counted from the arithmetic
# of the method with an FMA as two operations and rsqrt / division as one.
FORCE_OPS = {2: (47, 87), 3: (59, 127)}
CONT_OPS = {2: 37, 3: 46}

# Algorithmic HBM bytes of one force-pass launch (the packed form, which every
# workload here takes: one particle mass per fluid): each particle's own
# records read once (frozen position, {velocity, pressure}, viscous
# acceleration: 16 B each in the mixed form, but 12 B for the 3D frozen
# position, 32 B each in FP64), count and flags
# (5 B), the FP64 velocity read and written (2 x 8d B) and the kicked
# {velocity, pressure} record written; 4 B of neighbour index per pair; the
# colour record of near-interface particles.  Neighbour records gathered per
# pair are cache traffic.
FORCE_BYTES = {  # (per particle, per pair, per near-interface particle)
    (2, "mixed"): (101, 4, 16), (3, "mixed"): (113, 4, 16),
    (2, "fp64"): (165, 4, 32), (3, "fp64"): (181, 4, 32),
}

# Force-pass HBM traffic measured with rocprofv3 --pmc (FETCH_SIZE x 2 and
# WRITE_SIZE x 1, the scales a 1 GiB device copy reads) for the kernel code
# whose digest is recorded; any change of that code voids the figure.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_pass_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2503_16082_amd", "csrc", f)
                  for f in ("rsph_kernels.hip", "rsph_internal.h")]


def kernel_digest():
    """SHA-256 of the device code's sources (the kernels and the layout header
    they include) with comments and blank lines removed, so that a change of
    wording alone keeps a measurement (the sources hold no string that a
    comment marker could occur in, other than static_assert messages)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        src = open(path).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(l.rstrip() for l in src.splitlines() if l.strip()).encode())
    return h.hexdigest()


def recorded_traffic(workload, form):
    try:
        sha = kernel_digest()
        for line in open(TRAFFIC_FILE):
            f = line.split()
            if len(f) == 5 and f[0] == workload and f[1] == form and f[2] == sha:
                return float(f[3]) + float(f[4])
    except OSError:
        pass
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# profiling utilities: the copy reference of the byte counters, the traffic
# line of the force pass, and the kernel-trace summary tables of profiles/
# ---------------------------------------------------------------------------

COPY_BYTES = 1 << 30


def copy_probe():
    """One 1 GiB device-to-device copy: the reference by which FETCH_SIZE and
    WRITE_SIZE are scaled (run under rocprofv3 --pmc)."""
    import torch
    x = torch.ones(COPY_BYTES // 4, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}), flush=True)


def pmc_per_dispatch(csv_path, name_part, counter):
    """Counter value of every dispatch of the kernels whose name contains
    name_part (summed over the rows rocprofv3 writes for one dispatch)."""
    import csv
    import collections
    vals = collections.defaultdict(float)
    for row in csv.DictReader(open(csv_path)):
        if name_part in row["Kernel_Name"] and row["Counter_Name"] == counter:
            vals[int(row["Dispatch_Id"])] += float(row["Counter_Value"])
    return [vals[k] for k in sorted(vals)]


def active_mean(v):
    """Mean over the dispatches that did work (above a quarter of the largest:
    a launch cycle also issues substep launches that exit at once)."""
    top = max(v)
    act = [x for x in v if x > 0.25 * top]
    return sum(act) / len(act), len(act)


def pmc_traffic(args):
    f_csv, w_csv, cf_csv, cw_csv = args.pmc_traffic
    dim = 2 if args.workload in ("square2d", "droplet2d") else 3
    # the force pass in either record form (k_force<R, D> or k_force<R, D, packed>)
    kname = f"k_force<{'float' if args.precision == 'mixed' else 'double'}, {dim}"
    # the launches with work are those that write (a launch cycle also issues
    # substep launches that exit at once, which still fetch their slot-only
    # loads); the two runs dispatch the same sequence, so the fetch counts of
    # those same dispatches are averaged
    f_all = pmc_per_dispatch(f_csv, kname, "FETCH_SIZE")
    w_all = pmc_per_dispatch(w_csv, kname, "WRITE_SIZE")
    write, nw = active_mean(w_all)
    if len(f_all) == len(w_all):
        act = [k for k, x in enumerate(w_all) if x > 0.25 * max(w_all)]
        fetch, nf = sum(f_all[k] for k in act) / len(act), len(act)
    else:
        fetch, nf = active_mean(f_all)
    cf = max(pmc_per_dispatch(cf_csv, "copyBuffer", "FETCH_SIZE"))
    cw = max(pmc_per_dispatch(cw_csv, "copyBuffer", "WRITE_SIZE"))
    f_scale = COPY_BYTES / (cf * 1024.0)
    w_scale = COPY_BYTES / (cw * 1024.0)
    fetch_b = fetch * 1024.0 * f_scale
    write_b = write * 1024.0 * w_scale
    name = workload(args.workload)["name"]
    sha = kernel_digest()
    lines = []
    if os.path.exists(TRAFFIC_FILE):
        lines = [l for l in open(TRAFFIC_FILE).read().splitlines()
                 if not (len(l.split()) == 5 and l.split()[0] == name and l.split()[1] == args.precision)]
    lines.append(f"{name} {args.precision} {sha} {fetch_b:.0f} {write_b:.0f}")
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"workload": name, "form": args.precision, "kernel": kname, "dispatches": [nf, nw],
                      "fetch_kib": fetch, "write_kib": write, "copy_fetch_kib": cf, "copy_write_kib": cw,
                      "fetch_scale": f_scale, "write_scale": w_scale, "fetch_bytes": fetch_b,
                      "write_bytes": write_b}), flush=True)


def counter_summary(csv_paths):
    """Markdown table of the vector-memory and ALU utilisation of the pair
    kernels from rocprofv3 --pmc output (several runs, one counter group each;
    per kernel the dispatch with the most waves; busy fractions are counter
    totals per CU over the GPU-active cycles of one XCD)."""
    import collections
    import csv
    import re
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(list)))
    for path in csv_paths:
        for row in csv.DictReader(open(path)):
            k = re.sub(r"\(.*", "", row["Kernel_Name"]).replace("void ", "").replace("rsph::", "")
            per[path][(k, int(row["Dispatch_Id"]))][row["Counter_Name"]].append(float(row["Counter_Value"]))
    # the GPU agent's XCD and CU counts: GRBM_GUI_ACTIVE is summed over the XCDs
    n_xcc, cu = 1, 256
    agent_csv = os.path.join(os.path.dirname(csv_paths[0]), "run_agent_info.csv")
    if os.path.exists(agent_csv):
        for row in csv.DictReader(open(agent_csv)):
            if row.get("Vendor_Name") == "AMD" and row.get("Name", "").startswith("gfx"):
                n_xcc, cu = int(row["Num_Xcc"]), int(row["Cu_Count"])
    kern = collections.defaultdict(dict)
    for path, disp in per.items():
        best = {}
        for (k, d), cs in disp.items():
            waves = sum(cs.get("SQ_WAVES", [0.0]))
            key = sum(cs.get("GRBM_GUI_ACTIVE", [0.0])) if not waves else waves
            if k not in best or key > best[k][0]:
                best[k] = (key, cs)
        for k, (_, cs) in best.items():
            for c, v in cs.items():
                kern[k][c] = sum(v) / n_xcc if c == "GRBM_GUI_ACTIVE" else sum(v)
    out = ["| kernel | cycles per XCD | VALU busy | TA busy | TD busy | L1 hit | L2 hit | VALU instr/wave | VMEM rd/wave |",
           "|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(kern):
        c = kern[k]
        if not any(t in k for t in ("k_force", "k_continuity", "k_colour", "k_neighbours", "k_density",
                                    "k_advection", "k_shift")):
            continue
        gui = c.get("GRBM_GUI_ACTIVE", float("nan"))
        waves = c.get("SQ_WAVES", float("nan"))
        f = lambda x: f"{100 * x:.0f} %" if x == x else "-"
        tcp, req = c.get("TCP_TOTAL_CACHE_ACCESSES", float("nan")), c.get("TCP_TCC_READ_REQ", float("nan"))
        hit, miss = c.get("TCC_HIT_sum", float("nan")), c.get("TCC_MISS_sum", float("nan"))
        out.append(f"| `{k}` | {gui:.3e} | {f(c.get('SQ_ACTIVE_INST_VALU', float('nan')) / cu / gui)} | "
                   f"{f(c.get('TA_TA_BUSY', float('nan')) / cu / gui)} | {f(c.get('TD_TD_BUSY', float('nan')) / cu / gui)} | "
                   f"{f(1 - req / tcp)} | {f(hit / (hit + miss))} | {c.get('SQ_INSTS_VALU', float('nan')) / waves:.0f} | "
                   f"{c.get('SQ_INSTS_VMEM_RD', float('nan')) / waves:.1f} |")
    print("\n".join(out))


def trace_summary(db):
    """Markdown table of a rocprofv3 kernel-trace database: per kernel, the
    average over every dispatch and over the dispatches that did work."""
    import collections
    import re
    import sqlite3
    cur = sqlite3.connect(db).cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    ni, si, ei = cols.index("name"), cols.index("start"), cols.index("end")
    agg = collections.defaultdict(list)
    for r in cur.execute("select * from kernels").fetchall():
        agg[r[ni]].append((r[ei] - r[si]) / 1e3)
    tot = sum(sum(v) for v in agg.values())
    out = ["| kernel | calls | avg us (all) | total ms | share | active calls | avg us (active) |",
           "|---|---|---|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) / tot < 0.002:
            continue
        nm = re.sub(r"^void ", "", k).replace("rsph::", "")
        nm = re.sub(r"\((rsph::)?DevArrays.*", "", nm)
        act = [x for x in v if x > 0.25 * max(v)]
        out.append(f"| `{nm}` | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / 1e3:.3f} | "
                   f"{100 * sum(v) / tot:.1f}% | {len(act)} | {sum(act) / len(act):.2f} |")
    print("\n".join(out))


def workload(name):
    if name == "square2d":
        return WL.square_droplet_2d(n_side=200)
    if name == "droplet2d":
        return WL.static_droplet_2d(n_side=50)
    if name == "droplet3d":
        return WL.static_droplet_3d(n_side=64)
    if name == "impact3d":
        return WL.droplet_impact_3d()
    raise SystemExit(f"unknown workload {name}")


def run_gpu(w, precision, steps, warmup, timed_kernels, launch="graph"):
    """Warmup, then `steps` advection steps timed on the host clock (the
    step call returns after the stream is synchronised).  With timed_kernels,
    every launch of those kernels is bracketed by HIP events, which runs the
    cycles eagerly."""
    p = w["params"]
    s = rsph.System(p, precision=precision)
    s.set_launch_mode(launch)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    if warmup:
        s.step(warmup)
    o0 = s.observables()
    s.set_timing(timed_kernels)
    t0 = time.perf_counter()
    s.step(steps)
    t1 = time.perf_counter()
    timing = s.timing()
    o1 = s.observables()
    nnb = s.read("nnb")
    flags = s.read("flags").astype(np.int64)
    return s, {
        "seconds": t1 - t0,
        "substeps": int(o1["n_sub"] - o0["n_sub"]),
        "timing": timing,
        "pairs": float(nnb.sum()),
        "near_pairs": float(nnb[(flags & 2) != 0].sum()),
        "near": float(((flags & 2) != 0).sum()),
        "obs": o1,
        "momentum": (np.asarray(o0["momentum"], dtype=np.float64), np.asarray(o1["momentum"], dtype=np.float64)),
    }


def rate_errors(a, ref):
    """Single-evaluation error of an acceleration field against the oracle's:
    the normwise max_i |a_i - a_i^ref| / max_i |a_i^ref|, and the per-particle
    |a_i - a_i^ref| / |a_i^ref| over the particles with |a_i^ref| >= 1e-3 of the
    largest (its maximum and 99th percentile)."""
    d = np.linalg.norm(a - ref, axis=1)
    r = np.linalg.norm(ref, axis=1)
    big = r >= 1e-3 * r.max()
    rel = d[big] / r[big]
    return {"normwise": float(d.max() / r.max()), "per_particle_max": float(rel.max()),
            "per_particle_p99": float(np.percentile(rel, 99))}


def input_sample(w, n, seed=0):
    """Particles chosen from the inputs alone: every lattice particle whose
    unjittered site lies within 3h of the drop's or the pool's surface, or a
    random half of them if there are more than n / 2, plus n / 2 drawn at
    random from all particles."""
    rng = np.random.default_rng(seed)
    p = w["params"]
    h = p["dp"] * p.get("h_over_dp", 1.3)
    pos = w["pos"]
    near = np.abs(np.linalg.norm(pos - w["centre"], axis=1) - w["R"]) < 3 * h
    near |= np.abs(pos[:, 2] - w["pool_depth"]) < 3 * h
    near = np.where(near)[0]
    if len(near) > n // 2:
        near = rng.choice(near, n // 2, replace=False)
    return np.unique(np.concatenate([near, rng.choice(pos.shape[0], n // 2, replace=False)]))


def accel_error(w, precision, sample=4096):
    """Acceleration error of a GPU form against the FP64 oracle at the
    workload's initial state; above 300,000 particles the oracle evaluates a
    sample chosen from the inputs (input_sample)."""
    from oracle import oracle as O
    p = w["params"]
    s = rsph.System(p, precision=precision)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.eval_rates()
    acc = s.read("acc")
    pos, vel, rho, mass = s.read("pos"), s.read("vel"), s.read("rho"), s.read("mass")
    s.close()
    n = pos.shape[0]
    targets = None
    if n > 300000:
        targets = input_sample(w, sample)
        acc = acc[targets]
    ref = O.eval_rates(p, O.wrap(p, pos), vel, rho, mass, w["phase"], targets=targets)["acc"]
    out = rate_errors(acc, ref)
    out["particles"] = int(n if targets is None else len(targets))
    return out


def host_cpu():
    """CPU model and the OpenMP threads the oracle runs with."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return model, threads


def mem_available_bytes():
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemAvailable:"):
                return int(line.split()[1]) * 1024
    except OSError:
        pass
    return 0


# host bytes the oracle holds per particle while it steps: its frozen pair
# geometry (index, r_ij, |r_ij|, W, W' = 56 B per pair) and per-particle arrays
ORACLE_BYTES = {2: 56 * 30 + 600, 3: 56 * 100 + 800}


def cpu_baseline(w, min_seconds, max_steps=5000):
    """The FP64 oracle, untuned, on the host cores: a bounded sample of the same
    workload, its first advection steps.  Below a million particles whole
    advection steps are taken (five at a time) until at least min_seconds of
    host time have passed; above, exactly one advection step of the full
    workload, after checking that the host has the memory for it."""
    from oracle import oracle as O
    p = w["params"]
    n = w["pos"].shape[0]
    dim = p["dim"]
    model, threads = host_cpu()
    need = ORACLE_BYTES[dim] * n
    avail = mem_available_bytes()
    if avail and need > 0.8 * avail:
        return {"value": None, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
                "cpu_model": model,
                "sample": f"not run: the oracle needs ~{need / 2**30:.0f} GiB, {avail / 2**30:.0f} GiB available"}
    st = O.State(p, O.wrap(p, w["pos"]), w["vel"], w["phase"])
    chunk = 5 if n < 1_000_000 else 1
    outer_steps = 0
    t0 = time.perf_counter()
    while True:
        st.step(chunk)
        outer_steps += chunk
        dt = time.perf_counter() - t0
        if chunk == 1 or dt >= min_seconds or outer_steps >= max_steps:
            break
    return {
        "value": n * outer_steps / dt,
        "unit": "particle-steps/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": model,
        "sample": f"first {outer_steps} advection step(s) ({int(st.clock.n_sub)} substeps) of the "
                  f"same workload, all {n} particles, {dt:.1f} s on {threads} OpenMP threads",
        "particle_substeps_per_s": n * st.clock.n_sub / dt,
    }


# The oracle's CPU baselines of the benchmark set: (name, workload builder,
# advection steps timed).  The static droplet in full (200 steps), a 50-step
# window of the square droplet, one step of the 3D droplet and of the impact.
CPU_PLAN = [
    ("static_droplet_2d (2,500 particles, 200 steps)", lambda: WL.static_droplet_2d(n_side=50), 200),
    ("square_droplet_2d (40,000 particles, steps 1-50)", lambda: WL.square_droplet_2d(n_side=200), 50),
    ("static_droplet_3d (262,144 particles, 1 step)", lambda: WL.static_droplet_3d(n_side=64), 1),
    ("droplet_impact_3d (8,388,608 particles, 1 step)", lambda: WL.droplet_impact_3d(), 1),
]


def cpu_plan_leg(k):
    """One entry of CPU_PLAN timed on the oracle with the OpenMP threads of
    this process; one JSON line."""
    from oracle import oracle as O
    name, build, steps = CPU_PLAN[k]
    w = build()
    p = w["params"]
    n = w["pos"].shape[0]
    model, threads = host_cpu()
    need = ORACLE_BYTES[p["dim"]] * n
    avail = mem_available_bytes()
    if avail and need > 0.8 * avail:
        print(json.dumps({"workload": name, "threads": threads, "skipped": "host memory"}), flush=True)
        return
    st = O.State(p, O.wrap(p, w["pos"]), w["vel"], w["phase"])
    t0 = time.perf_counter()
    st.step(steps)
    dt = time.perf_counter() - t0
    print(json.dumps({"workload": name, "particles": n, "threads": threads, "cpu_model": model, "steps": steps,
                      "substeps": int(st.clock.n_sub), "seconds": dt, "particle_steps_per_s": n * steps / dt,
                      "particle_substeps_per_s": n * st.clock.n_sub / dt}), flush=True)


def cpu_baselines(single_max):
    """Every entry of CPU_PLAN on all of the host's threads, and the entries
    up to single_max on one thread (the plain figure), each in a child
    process that sets OMP_NUM_THREADS before the oracle loads."""
    import subprocess
    runs = [(k, None) for k in range(len(CPU_PLAN))] + [(k, 1) for k in range(min(single_max + 1, len(CPU_PLAN)))]
    for k, threads in runs:
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = str(threads)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-plan-leg", str(k)], env=env,
                           capture_output=True, text=True)
        sys.stdout.write(r.stdout)
        sys.stdout.flush()
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise SystemExit(r.returncode)


def served_leg(args, log_jobs=False):
    """Served form on the mixed droplet stream: the saturated job rate is taken
    from a probe batch that arrives all at once; the full stream then arrives
    as a Poisson process at 0.8 of that rate into a pool with a fixed HBM
    budget.  Returns the summary."""
    from paper_2503_16082_amd import serve
    prec = rsph.MIXED if args.precision == "mixed" else rsph.FP64
    descs = WL.served_mix(n_jobs=args.jobs, seed=0)
    budget = int(args.budget_gb * (1 << 30))
    probe = descs[:args.probe_jobs]
    # probe jobs as long as the stream's: admission costs (pool repack, graph
    # capture) then weigh as much per step as in the stream.  The saturated
    # job rate is the probe's particle-step rate over the stream's mean work
    # per job, so that the probe's own job sizes do not set it.
    probe_steps = args.probe_steps or args.steps_per_job
    cap = args.max_steps_per_tick
    ps = serve.serve(probe, steps_per_job=probe_steps, rate_hz=None, budget_bytes=budget, precision=prec,
                     max_steps_per_tick=cap, max_admits_per_tick=args.max_admits_per_tick)
    n_side = [max(3, int(round(math.sqrt(d["n"])))) for d in descs]
    work_per_job = float(np.mean([k * k for k in n_side])) * args.steps_per_job
    rate_sat = ps["particle_steps_per_s"] / work_per_job
    log(f"probe: {ps['jobs']} jobs x {probe_steps} steps in {ps['wall_s']:.2f}s -> saturated "
        f"{rate_sat:.3f} jobs/s at {args.steps_per_job} steps per job")
    rate = 0.8 * rate_sat
    out = serve.serve(descs, steps_per_job=args.steps_per_job, rate_hz=rate, budget_bytes=budget,
                      precision=prec, log=log if log_jobs else None, max_steps_per_tick=cap,
                      max_admits_per_tick=args.max_admits_per_tick)
    out.update({"arrival_rate_hz": rate, "saturated_job_rate_hz": rate_sat, "hbm_budget_bytes": budget,
                "jobs_in_stream": args.jobs, "steps_per_job": args.steps_per_job,
                "particles_per_job": "log-uniform 2,000-200,000", "form": args.precision})
    return out


def served(args):
    """--workload served: the served leg alone, as its own JSON line."""
    out = served_leg(args, log_jobs=True)
    prec = rsph.MIXED if args.precision == "mixed" else rsph.FP64
    line = {
        "metric": "served particle-steps/s with p50/p99 per-step latency",
        "value": out["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32" if prec == rsph.MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": "served_mix", "jobs": args.jobs, "steps_per_job": args.steps_per_job,
                   "particles_per_job": "log-uniform 2,000-200,000", "arrival_rate_hz": out["arrival_rate_hz"],
                   "hbm_budget_bytes": out["hbm_budget_bytes"], "form": args.precision,
                   "max_steps_per_tick": args.max_steps_per_tick,
                   "max_admits_per_tick": args.max_admits_per_tick},
    }
    for k in ("step_latency_p50_ms", "step_latency_p99_ms", "tick_latency_p50_ms", "tick_latency_p99_ms",
              "step_interval_p50_ms", "step_interval_p99_ms", "turnaround_p50_s", "max_queue_depth",
              "wall_s", "saturated_job_rate_hz"):
        line[k] = out[k]
    line["jobs_done"] = out["jobs"]
    print(json.dumps(line), flush=True)


def roofline_block(gbs, tflops, peak_tf, working_set):
    """The roofline object of the force pass. Its bound is the unit whose peak the
    launch uses the larger share of. For HBM that share is the algorithmic bytes
    over the launch time, and it counts only when the working set exceeds the
    Infinity Cache; otherwise the bytes come from on-chip caches. For the vector
    ALU it is the counted operations over the launch time. Both shares are kept
    beside the chosen one."""
    hbm_frac = gbs / PEAK_HBM_GBS
    alu_frac = tflops / peak_tf
    exceeds = working_set > MALL_BYTES
    if exceeds and hbm_frac >= alu_frac:
        head = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": hbm_frac}
    else:
        head = {"bound": "alu", "achieved": tflops, "peak": peak_tf, "unit": "TFLOP/s", "frac": alu_frac}
    head.update({
        "hbm_achieved_gbs": gbs, "hbm_peak_gbs": PEAK_HBM_GBS, "hbm_frac": hbm_frac,
        "alu_achieved_tflops": tflops, "alu_peak_tflops": peak_tf, "alu_frac": alu_frac,
        "working_set_exceeds_mall": exceeds,
    })
    return head


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed advection steps (default: 20 for the 8.4M-particle impact, 40 for the 3D "
                         "static droplet, 500 for the 2D workloads)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed advection steps first (default: 3, 2, 10)")
    ap.add_argument("--workload", default="impact3d",
                    choices=["impact3d", "square2d", "droplet2d", "droplet3d", "served"])
    ap.add_argument("--jobs", type=int, default=256, help="served: jobs in the stream")
    ap.add_argument("--steps-per-job", type=int, default=200, help="served: advection steps per job")
    ap.add_argument("--budget-gb", type=float, default=0.5, help="served: pool HBM budget")
    ap.add_argument("--probe-jobs", type=int, default=24, help="served: jobs of the saturation probe")
    ap.add_argument("--probe-steps", type=int, default=None,
                    help="served: steps per probe job (default: the stream's steps per job)")
    ap.add_argument("--max-admits-per-tick", type=int, default=0,
                    help="served: most admissions between two ticks (0: as many as the budget holds)")
    ap.add_argument("--max-steps-per-tick", type=int, default=4,
                    help="served: most advection steps a job takes per scheduler tick (1: lockstep)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true", help="leave the served leg out of the bench line")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="host time of the oracle sample below a million particles (whole advection steps, "
                         "at least this long)")
    ap.add_argument("--no-accel-check", action="store_true",
                    help="skip the single-evaluation acceleration check against the oracle")
    ap.add_argument("--copy-probe", action="store_true", help="1 GiB device copy (counter reference)")
    ap.add_argument("--cpu-baselines", action="store_true",
                    help="the oracle on the host's cores over the benchmark set (no GPU): one JSON line each")
    ap.add_argument("--cpu-single-max", type=int, default=2,
                    help="--cpu-baselines: also run the first entries up to this index on one thread")
    ap.add_argument("--cpu-plan-leg", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--pmc-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the force-pass traffic line of --workload/--precision from rocprofv3 --pmc output")
    ap.add_argument("--trace-summary", metavar="DB", help="markdown table of a rocprofv3 kernel-trace database")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="markdown table of pair-kernel utilisation from rocprofv3 --pmc output")
    args = ap.parse_args()
    if args.cpu_plan_leg is not None:
        cpu_plan_leg(args.cpu_plan_leg)
        return
    if args.cpu_baselines:
        cpu_baselines(args.cpu_single_max)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.pmc_traffic:
        pmc_traffic(args)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the method's hot path is single-GPU here; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "served":
        served(args)
        return
    steps0, warm0 = {"droplet3d": (40, 2), "impact3d": (20, 3)}.get(args.workload, (500, 10))
    args.steps = steps0 if args.steps is None else args.steps
    args.warmup = warm0 if args.warmup is None else args.warmup
    w = workload(args.workload)
    n = w["pos"].shape[0]
    dim = w["params"]["dim"]
    prec = rsph.MIXED if args.precision == "mixed" else rsph.FP64
    log(f"workload {w['name']} n={n} precision={args.precision} steps={args.steps} warmup={args.warmup}")

    # the timed region: graph replays, no per-launch events
    s, r = run_gpu(w, prec, args.steps, args.warmup, [])
    s.close()
    secs = r["seconds"]
    value = n * args.steps / secs
    log(f"gpu {secs:.3f}s -> {value:.3e} particle-steps/s, {r['substeps'] / args.steps:.2f} substeps/step")
    # the force-pass duration: the same steps again, every force launch
    # bracketed by HIP events on the system's stream (the events lengthen the
    # step, so they stay out of the timed region)
    s, rt = run_gpu(w, prec, args.steps, args.warmup, ["force"])
    s.close()
    f_launch, f_ms = rt["timing"]["force"]
    e_launch, e_ms = rt["timing"]["event_floor"]
    floor_ms = e_ms / max(e_launch, 1)
    # launches in which the system was inside an advection step, each bracketed
    # by HIP events recorded by its own dispatch
    f_avg_ms = f_ms / max(f_launch, 1)
    bulk_ops, surf_ops = FORCE_OPS[dim]
    ops = rt["pairs"] * bulk_ops + rt["near_pairs"] * surf_ops
    tflops = ops / (f_avg_ms * 1e-3) / 1e12
    peak_tf = PEAK_TFLOPS["f32" if prec == rsph.MIXED else "f64"]
    per_p, per_pair, per_near = FORCE_BYTES[(dim, args.precision)]
    algo_bytes = n * per_p + rt["pairs"] * per_pair + rt["near"] * per_near
    gbs = algo_bytes / (f_avg_ms * 1e-3) / 1e9
    log(f"force launches={f_launch} avg={f_avg_ms * 1e3:.1f}us bytes/launch={algo_bytes:.3e} -> {gbs:.1f} GB/s; "
        f"ops/launch={ops:.3e} -> {tflops:.2f} TFLOP/s")

    extra = {}
    if prec == rsph.MIXED and not args.no_fp64_compare:
        try:
            s64, r64 = run_gpu(w, rsph.FP64, args.steps, args.warmup, [])
            s64.close()
            v64 = n * args.steps / r64["seconds"]
            s64, rt64 = run_gpu(w, rsph.FP64, args.steps, args.warmup, ["force"])
            s64.close()
            l64, m64 = rt64["timing"]["force"]
            extra["fp64_gpu_value"] = v64
            extra["mixed_over_fp64"] = value / v64
            extra["fp64_substeps_per_step"] = r64["substeps"] / args.steps
            extra["fp64_force_avg_us"] = m64 / max(l64, 1) * 1e3
            log(f"fp64 gpu {r64['seconds']:.3f}s -> {v64:.3e} particle-steps/s, mixed/fp64 = {value / v64:.2f}")
        except rsph.RsphError as e:  # a health check of the FP64 run: reported, not timed
            extra["fp64_gpu_value"] = None
            extra["fp64_fault"] = str(e)
            log(f"fp64 gpu run stopped: {e}")
    if not args.no_accel_check:
        try:
            err = accel_error(w, prec)
            extra["accel_err_vs_fp64_oracle"] = err["normwise"]
            extra["accel_err_per_particle_p99"] = err["per_particle_p99"]
            extra["accel_err_per_particle_max"] = err["per_particle_max"]
            extra["accel_err_particles"] = err["particles"]
            if prec == rsph.MIXED:
                e64 = accel_error(w, rsph.FP64)
                extra["fp64_gpu_accel_err_vs_oracle"] = e64["normwise"]
            log(f"accel error vs oracle: {err}")
        except Exception as e:  # the oracle is a checker, not the product
            log(f"accel error check skipped: {e}")

    # the served leg and the CPU baseline are reported beside the measured
    # value: an error in either is recorded in the line, which is still printed
    srv = None
    if not args.no_served:
        try:
            srv = served_leg(args)
            log(f"served: {srv['particle_steps_per_s']:.3e} particle-steps/s, p50 {srv['step_latency_p50_ms']:.2f} "
                f"ms, p99 {srv['step_latency_p99_ms']:.2f} ms per step")
        except Exception as e:
            extra["served_error"] = f"{type(e).__name__}: {e}"
            log(f"served leg failed: {e}")

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(w, args.cpu_seconds)
            log(f"cpu baseline {cpu}")
        except Exception as e:
            extra["cpu_baseline_error"] = f"{type(e).__name__}: {e}"
            log(f"cpu baseline failed: {e}")

    # the force pass streams from HBM only when the workload's working set
    # exceeds the Infinity Cache
    working_set = n * (1300 if dim == 3 else 800)
    roof = roofline_block(gbs, tflops, peak_tf, working_set)
    roof.update({
        "kernel": "force pass (k_force)",
        "traffic": recorded_traffic(w["name"], args.precision),
        "algorithmic_bytes_per_launch": algo_bytes,
        "ops_per_launch": ops,
        "avg_launch_us": f_avg_ms * 1e3,
        "launches": f_launch,
        "empty_kernel_event_us": floor_ms * 1e3,
    })
    line = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == rsph.MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": w["name"],
            "particles": n,
            "dim": dim,
            "form": args.precision,
            "step": "one advection step with all its acoustic substeps",
            "parallelism": "single GPU",
        },
        "particle_substeps_per_s": n * r["substeps"] / secs,
        "substeps_per_step": r["substeps"] / args.steps,
        # total momentum over the timed steps: |P(end) - P(start)|, and, for the
        # impact (which carries the drop's momentum), that relative to |P(start)|
        "momentum_change": float(np.linalg.norm(r["momentum"][1] - r["momentum"][0])),
        "momentum_drift": (float(np.linalg.norm(r["momentum"][1] - r["momentum"][0])
                                 / np.linalg.norm(r["momentum"][0]))
                           if args.workload == "impact3d" else None),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if srv is not None:
        line["served_particle_steps_per_s"] = srv["particle_steps_per_s"]
        line["served_step_latency_p50_ms"] = srv["step_latency_p50_ms"]
        line["served_step_latency_p99_ms"] = srv["step_latency_p99_ms"]
        line["served"] = {k: srv[k] for k in (
            "jobs", "jobs_in_stream", "steps_per_job", "particles_per_job", "form", "arrival_rate_hz",
            "saturated_job_rate_hz", "hbm_budget_bytes", "wall_s", "tick_latency_p50_ms", "tick_latency_p99_ms",
            "step_interval_p50_ms", "step_interval_p99_ms", "turnaround_p50_s", "max_queue_depth")}
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
