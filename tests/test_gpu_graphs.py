"""Launch cycles replayed from captured HIP graphs against the same cycles
launched kernel by kernel.

Both modes launch the same kernels with the same arguments, so every replay
must give the eager result bit for bit.  Each replay is checked, with eager
work (observable reductions, field reads, synchronisations) between replays.
"""
import sys

import numpy as np
import pytest

from paper_2503_16082_amd import workloads as WL

pytestmark = pytest.mark.gpu

rsph = pytest.importorskip("paper_2503_16082_amd.rsph")

KEYS = ["pos", "vel", "rho", "drho"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fields(s):
    return {k: s.read(k) for k in KEYS}


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_match_eager(dim, precision):
    if dim == 2:
        w = WL.static_droplet_2d(n_side=40, R=0.2, seed=11)
    else:
        w = WL.static_droplet_3d(n_side=16, seed=11)
    say(f"graph vs eager dim={dim} precision={precision} n={w['pos'].shape[0]}")
    runs = {}
    for mode in ("eager", "graph"):
        s = rsph.System(w["params"], precision=precision)
        s.set_launch_mode(mode)
        s.set_particles(w["pos"], w["vel"], w["phase"])
        seq = []
        for _ in range(4):
            s.step(1)
            o = s.observables()  # eager reduction kernels between replays
            seq.append((fields(s), o["n_sub"], o["t"]))
        runs[mode] = seq
        s.close()
    for k, (a, b) in enumerate(zip(runs["eager"], runs["graph"])):
        assert a[1] == b[1] and a[2] == b[2], k
        for f in KEYS:
            assert np.array_equal(a[0][f], b[0][f]), (k, f)


def test_graph_pool_layout_changes_and_timing():
    """Admission and release change the pool layout (new graphs are captured);
    a timed stretch runs eagerly in between.  Every job equals the same job
    stepped eagerly on its own."""
    ws = [WL.oscillating_ellipse_2d(2500, 1.3, 1000.0, 1.0, seed=21),
          WL.oscillating_ellipse_2d(4900, 1.2, 100.0, 0.7, seed=22),
          WL.static_droplet_2d(n_side=36, seed=23)]

    def alone(w, steps):
        s = rsph.System(w["params"], precision=1)
        s.set_launch_mode("eager")
        s.set_particles(w["pos"], w["vel"], w["phase"])
        s.step(steps)
        out = fields(s)
        s.close()
        return out

    pool = rsph.Pool(2, precision=1)
    a = pool.admit(ws[0]["params"], ws[0]["pos"], ws[0]["vel"], ws[0]["phase"])
    a.set_launch_mode("graph")
    b = pool.admit(ws[1]["params"], ws[1]["pos"], ws[1]["vel"], ws[1]["phase"])
    pool.step([a, b], [2, 1])
    a.set_timing(["force"])  # timed launches are eager
    pool.step([a, b], [1, 2])
    a.set_timing([])
    pool.release(b)
    c = pool.admit(ws[2]["params"], ws[2]["pos"], ws[2]["vel"], ws[2]["phase"])
    pool.step([a, c], [1, 2])
    pool.step([a, c], [1, 1])
    ref_a, ref_c = alone(ws[0], 5), alone(ws[2], 3)
    got_a, got_c = fields(a), fields(c)
    for f in KEYS:
        assert np.array_equal(got_a[f], ref_a[f]), f
        assert np.array_equal(got_c[f], ref_c[f]), f
    pool.close()
    say("pool graph/eager parity ok")


def test_invalid_launch_mode():
    w = WL.static_droplet_2d(n_side=20, seed=24)
    s = rsph.System(w["params"])
    r = rsph.lib().rsph_set_launch_mode(s.h, 7)
    assert rsph.STATUS[r] == "EINVAL"
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_timing_counts_only_launches_with_work(dim):
    """A system created where an earlier one freed its memory: the timed force
    and continuity launches that count are exactly the substeps taken."""
    w = WL.static_droplet_2d(n_side=40, seed=31) if dim == 2 else WL.static_droplet_3d(n_side=16, seed=31)
    first = rsph.System(w["params"], precision=1)
    first.set_particles(w["pos"], w["vel"], w["phase"])
    first.step(2)
    first.close()
    s = rsph.System(w["params"], precision=1)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(1)
    n0 = s.observables()["n_sub"]
    s.set_timing(["force", "continuity"])
    s.step(3)
    t = s.timing()
    dn = s.observables()["n_sub"] - n0
    say(f"timing dim={dim}: substeps {dn}, force launches {t['force'][0]}, continuity {t['continuity'][0]}")
    assert t["force"][0] == dn
    assert t["continuity"][0] == dn
    s.close()
