"""The served form against the oracle, and its fault isolation.

Pools of several systems find each lane's system through the per-wave table
(a pool of one system skips it), so the pooled jobs are compared here with the
FP64 oracle directly, in both forms: a pool of four jobs of different sizes,
density ratios and surface tensions, each stepped by its own count.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_16082_amd import workloads as WL

pytestmark = pytest.mark.gpu

rsph = pytest.importorskip("paper_2503_16082_amd.rsph")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


def jobs():
    return [
        WL.oscillating_ellipse_2d(2500, 1.3, 1000.0, 1.0, seed=1),
        WL.oscillating_ellipse_2d(6400, 1.2, 10.0, 0.7, seed=2),
        WL.oscillating_ellipse_2d(3600, 1.45, 100.0, 1.8, seed=3),
        WL.oscillating_drop_2d(n_side=40, ratio=1000.0, V0=1.0, gamma=1.0, seed=4),
    ]


# trajectory tolerance after a few advection steps (normwise velocity and
# density deviation, position in units of dp): FP64 against FP64 differs by
# summation order only; the mixed form's pair sums carry FP32 rounding (1e-5
# per evaluation) into the state
TRAJ = {0: (1e-9, 1e-10), 1: (1e-4, 1e-4)}


@pytest.mark.parametrize("precision", [0, 1])
def test_pooled_jobs_match_the_oracle(precision):
    ws = jobs()
    steps = [3, 2, 3, 4]
    pool = rsph.Pool(2, precision=precision)
    members = [pool.admit(w["params"], w["pos"], w["vel"], w["phase"]) for w in ws]
    pool.step(members, steps)
    tol_v, tol_x = TRAJ[precision]
    for k, (w, m, n) in enumerate(zip(ws, members, steps)):
        p = w["params"]
        st = O.State(p, w["pos"], w["vel"], w["phase"])
        st.step(n)
        o = m.observables()
        assert o["n_outer"] == n and o["health"] == 0
        if precision == 0:
            assert o["n_sub"] == st.clock.n_sub
            assert o["t"] == pytest.approx(st.clock.t, rel=1e-12)
        else:
            assert abs(o["n_sub"] - st.clock.n_sub) <= max(1, n)
        rho0 = np.asarray(p["rho0"])[w["phase"]]
        ev = normwise(m.read("vel"), st.vel)
        er = normwise(m.read("rho") - rho0, st.rho - rho0)
        dpos = m.read("pos") - O.wrap(p, st.pos)
        dpos -= np.round(dpos)
        ex = np.abs(dpos).max() / p["dp"]
        say(f"pooled job {k} (n={len(w['pos'])}, {n} steps, precision {precision}): "
            f"vel {ev:.2e} rho {er:.2e} pos {ex:.2e} dp")
        assert ev < tol_v and er < tol_v and ex < tol_x
    # one evaluation of every rate of a pool member at its current state,
    # against the oracle at the same state
    m, w = members[2], ws[2]
    m.eval_rates()
    pos, vel, rho, mass = (m.read(f) for f in ("pos", "vel", "rho", "mass"))
    ref = O.eval_rates(w["params"], O.wrap(w["params"], pos), vel, rho, mass, w["phase"])
    e = normwise(m.read("acc"), ref["acc"])
    say(f"pooled member rates: acc {e:.2e}")
    assert e <= (1e-12 if precision == 0 else 1e-5)
    pool.close()


def test_serving_loop_isolates_a_faulted_job():
    """A request loop whose stream holds a job with a 1e30 velocity (its
    acoustic step collapses at its first advection step; every kernel exits
    normally): that job is released and reported with its health bits, and
    every other job finishes with the result it has alone."""
    from paper_2503_16082_amd import serve
    descs = WL.served_mix(n_jobs=5, seed=4, n_min=2000, n_max=6000)

    def builder(d):
        w = serve.build_job(d)
        if d["job"] == 2:
            w["vel"] = w["vel"].copy()
            w["vel"][0, 0] = 1e30
        return w

    out = serve.serve(descs, steps_per_job=3, rate_hz=None, budget_bytes=0, precision=1,
                      keep_results=True, builder=builder)
    say({k: v for k, v in out.items() if k != "results"})
    assert out["jobs"] == 4 and out["jobs_failed"] == 1
    assert list(out["failed_health"]) == [2] and out["failed_health"][2] & 32
    for k in (0, 1, 3, 4):
        w = serve.build_job(descs[k])
        s = rsph.System(w["params"], precision=1)
        s.set_particles(w["pos"], w["vel"], w["phase"])
        s.step(3)
        for f in ("pos", "vel", "rho"):
            assert np.array_equal(out["results"][k][f], s.read(f)), (k, f)
        s.close()
