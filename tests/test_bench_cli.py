"""bench.py without a GPU: the single-GPU contract, and the profiling utilities
that turn rocprofv3 output into the summaries and the traffic figure."""
import csv
import os
import sqlite3
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import numpy as np  # noqa: E402
import pytest  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_trace_summary_table(tmp_path, capsys):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = []
    t = 0
    for k in range(10):  # 6 active force launches of 10 us, 4 idle ones of 1 us
        d = 10000 if k < 6 else 1000
        rows.append(("void rsph::k_force<float, 2>(rsph::DevArrays)", t, t + d))
        t += d + 500
    rows.append(("rsph::k_dt_substep(rsph::DevArrays, long, int)", t, t + 3000))
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    bench.trace_summary(str(db))
    out = capsys.readouterr().out.splitlines()
    force = [l for l in out if "k_force<float, 2>" in l][0].split("|")
    cells = [c.strip() for c in force]
    assert cells[2] == "10"                    # calls
    assert float(cells[3]) == (6 * 10 + 4 * 1) / 10  # avg over all dispatches, us
    assert cells[6] == "6"                     # active calls
    assert float(cells[7]) == 10.0             # active average
    assert any("k_dt_substep" in l for l in out)


def write_counters(path, kernel, counter, per_dispatch):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, v in enumerate(per_dispatch):
            # two rows per dispatch, as for a counter summed over instances
            for half in (0.5, 0.5):
                w.writerow({"Dispatch_Id": d + 1, "Kernel_Name": kernel, "Counter_Name": counter,
                            "Counter_Value": v * half})


def test_pmc_traffic_line(tmp_path, monkeypatch):
    kern = "void rsph::k_force<float, 2>(rsph::DevArrays)"
    f_csv, w_csv = tmp_path / "f.csv", tmp_path / "w.csv"
    cf_csv, cw_csv = tmp_path / "cf.csv", tmp_path / "cw.csv"
    write_counters(f_csv, kern, "FETCH_SIZE", [4000.0, 4000.0, 10.0])   # KiB; the last is idle
    write_counters(w_csv, kern, "WRITE_SIZE", [1000.0, 1000.0, 5.0])
    copy = "__amd_rocclr_copyBuffer"
    write_counters(cf_csv, copy, "FETCH_SIZE", [(1 << 20) / 2])  # reads half of 1 GiB in KiB
    write_counters(cw_csv, copy, "WRITE_SIZE", [1 << 20])
    traffic = tmp_path / "traffic.txt"
    traffic.write_text("square_droplet_2d mixed oldsha 1 2\nother_workload mixed sha 3 4\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    args = types.SimpleNamespace(pmc_traffic=[str(f_csv), str(w_csv), str(cf_csv), str(cw_csv)],
                                 workload="square2d", precision="mixed")
    bench.pmc_traffic(args)
    lines = traffic.read_text().splitlines()
    assert "other_workload mixed sha 3 4" in lines
    mine = [l.split() for l in lines if l.startswith("square_droplet_2d mixed")]
    assert len(mine) == 1
    assert mine[0][2] == bench.kernel_digest()
    assert float(mine[0][3]) == 4000.0 * 1024 * 2.0   # fetch scaled by the copy's factor 2
    assert float(mine[0][4]) == 1000.0 * 1024 * 1.0
    assert bench.recorded_traffic("square_droplet_2d", "mixed") == 4000.0 * 1024 * 2.0 + 1000.0 * 1024


def test_pmc_traffic_pairs_fetch_with_the_launches_that_write(tmp_path, monkeypatch):
    # an idle substep launch still fetches its slot-only loads (here 1500 KiB,
    # above a quarter of the largest) but writes nothing: it is left out
    kern = "void rsph::k_force<float, 3, true, false>(rsph::DevArrays)"
    f_csv, w_csv = tmp_path / "f.csv", tmp_path / "w.csv"
    cf_csv, cw_csv = tmp_path / "cf.csv", tmp_path / "cw.csv"
    write_counters(f_csv, kern, "FETCH_SIZE", [4000.0, 1500.0, 4000.0])
    write_counters(w_csv, kern, "WRITE_SIZE", [1000.0, 0.0, 1000.0])
    write_counters(cf_csv, "__amd_rocclr_copyBuffer", "FETCH_SIZE", [(1 << 20) / 2])
    write_counters(cw_csv, "__amd_rocclr_copyBuffer", "WRITE_SIZE", [1 << 20])
    traffic = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    args = types.SimpleNamespace(pmc_traffic=[str(f_csv), str(w_csv), str(cf_csv), str(cw_csv)],
                                 workload="impact3d", precision="mixed")
    bench.pmc_traffic(args)
    line = traffic.read_text().split()
    assert line[0] == "droplet_impact_3d" and float(line[3]) == 4000.0 * 1024 * 2.0


def test_cpu_plan_leg_prints_a_baseline_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-plan-leg", "0"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    import json
    d = json.loads(r.stdout.strip().splitlines()[-1])
    assert d["particles"] == 2500 and d["steps"] == 200 and d["substeps"] >= 200
    assert d["particle_steps_per_s"] > 0 and d["threads"] >= 1 and d["cpu_model"]


def test_bench_line_keys_documented():
    # the keys of the benchmark line are produced by the default mode
    src = open(os.path.join(ROOT, "bench.py")).read()
    for key in ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]:
        assert f'"{key}"' in src, key


def test_served_and_error_keys_in_the_default_line():
    src = open(os.path.join(ROOT, "bench.py")).read()
    for key in ["served_step_latency_p50_ms", "served_step_latency_p99_ms", "served_particle_steps_per_s",
                "particle_substeps_per_s", "accel_err_per_particle_p99", "fp64_gpu_value", "cpu_model"]:
        assert f'"{key}"' in src, key
    assert 'default="impact3d"' in src


def test_rate_errors_normwise_and_per_particle():
    import bench
    ref = np.array([[1.0, 0.0], [0.0, 2.0], [1e-6, 0.0], [3.0, 4.0]])
    a = ref.copy()
    a[0, 0] += 1e-3        # 1e-3 relative to its own |a| = 1
    a[2, 0] += 1e-7        # a tiny acceleration: below 1e-3 of the max, not counted per particle
    e = bench.rate_errors(a, ref)
    assert e["normwise"] == pytest.approx(1e-3 / 5.0)
    assert e["per_particle_max"] == pytest.approx(1e-3)
    assert 0 < e["per_particle_p99"] <= 1e-3


def test_impact_sample_is_chosen_from_the_inputs():
    import bench
    from paper_2503_16082_amd import workloads as WL
    w = WL.droplet_impact_3d(n_per_unit=8)
    t = bench.input_sample(w, 1000)
    assert 900 <= len(t) <= 1000 and len(np.unique(t)) == len(t)
    h = 1.3 / 8
    pos = w["pos"][t]
    near = (np.abs(np.linalg.norm(pos - w["centre"], axis=1) - w["R"]) < 3 * h) | (
        np.abs(pos[:, 2] - w["pool_depth"]) < 3 * h)
    assert near.sum() >= 500
    assert np.array_equal(t, bench.input_sample(w, 1000))


def test_roofline_bound_is_the_larger_share():
    import bench
    big, small = 10 * bench.MALL_BYTES, bench.MALL_BYTES // 2
    # HBM share 0.5 against ALU 0.25, working set beyond the MALL: HBM-bound
    r = bench.roofline_block(4000.0, 19.65, 78.6, big)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["frac"] - 0.5) < 1e-12
    # the same rates on a cache-resident working set: the HBM share is no evidence
    r = bench.roofline_block(4000.0, 19.65, 78.6, small)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and abs(r["frac"] - 0.25) < 1e-12
    # ALU share 0.31 against HBM 0.22: ALU-bound, both shares kept
    r = bench.roofline_block(1767.0, 24.24, 78.6, big)
    assert r["bound"] == "alu" and abs(r["frac"] - 24.24 / 78.6) < 1e-12
    assert abs(r["hbm_frac"] - 1767.0 / 8000.0) < 1e-12 and r["working_set_exceeds_mall"]


def test_kernel_digest_ignores_comments_only(tmp_path, monkeypatch):
    import bench
    a = tmp_path / "a.hip"
    b = tmp_path / "b.h"
    a.write_text("// one wording\nint f(int x) { return x + 1; }  // trailing\n/* block\n comment */\n")
    b.write_text("constexpr int k = 4;\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a), str(b)])
    d0 = bench.kernel_digest()
    a.write_text("// another wording\n\nint f(int x) { return x + 1; }\n")
    assert bench.kernel_digest() == d0
    a.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_digest() != d0
    a.write_text("int f(int x) { return x + 1; }\n")
    b.write_text("constexpr int k = 8;\n")
    assert bench.kernel_digest() != d0
