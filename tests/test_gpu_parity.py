"""Parity of the HIP library (through its C-ABI) with the FP64 CPU oracle.

Binning and neighbour sets are compared bit-exactly; floating-point rates are
compared normwise: e = max_i |x_i - x_i^oracle| / max_i |x_i^oracle|, with
e <= 1e-12 for the FP64 form (summation order differs) and e <= 1e-5 for the
mixed form (FP32 pair arithmetic).
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_16082_amd import workloads as WL

pytestmark = pytest.mark.gpu

rsph = pytest.importorskip("paper_2503_16082_amd.rsph")

TOL = {0: 1e-12, 1: 1e-5}
FIELDS = ["gradC", "acc", "acc_p", "acc_s", "acc_v", "drho", "B", "dr", "sigma"]
GPU_NAME = {"drho": "rate_drho"}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a).max())


def perturbed_state(w, seed=1, vscale=None, drho=0.01):
    """Workload state with random velocities and density perturbations so that
    every term of the method is exercised."""
    p = dict(w["params"])
    d = p["dim"]
    rng = np.random.default_rng(seed)
    n = w["pos"].shape[0]
    pos = O.wrap(p, w["pos"])
    rho0 = np.asarray(p["rho0"])[w["phase"]]
    if vscale is None:
        vscale = 0.1 * p["c0"]
    vel = vscale * rng.normal(size=(n, d))
    rho = rho0 * (1.0 + drho * rng.normal(size=n))
    mass = rho0 / O.sigma0(d, p["dp"] * p.get("h_over_dp", 1.3), p["dp"])
    return p, pos, vel, rho, mass, w["phase"]


def gpu_rates(p, pos, vel, rho, mass, phase, precision):
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, vel, phase, mass=mass, rho=rho)
    s.eval_rates()
    out = {k: s.read(GPU_NAME.get(k, k)) for k in FIELDS}
    out["nnb"] = s.read("nnb")
    s.close()
    return out


def per_particle(a, b):
    """|a_i - b_i| / |b_i| over the particles with |b_i| >= 1e-3 max |b|: the
    99th percentile and the maximum."""
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    nb = np.linalg.norm(b, axis=1)
    big = nb >= 1e-3 * nb.max()
    rel = np.linalg.norm(a - b, axis=1)[big] / nb[big]
    return float(np.percentile(rel, 99)), float(rel.max())


# per-particle relative acceleration error |a_i - a_i^ref| / |a_i^ref| over the
# particles with |a_i^ref| >= 1e-3 of the largest, 99th percentile.  The 1e-5
# bound of the mixed form is stated normwise (TOL): a particle near
# equilibrium sums FP32 pair terms far larger than its net acceleration, so its
# own relative error is that much larger; its 99th percentile is held to 5e-5
# (measured up to 1.2e-5 on the 3D droplet after 10 advection steps)
TOL_P99 = {0: 1e-10, 1: 5e-5}


def compare_rates(g, ref, precision, label, targets=None):
    tol = TOL[precision]
    errs = {}
    for k in FIELDS:
        a = g[k] if targets is None else g[k][targets]
        errs[k] = normwise(a, ref[k])
    acc = g["acc"] if targets is None else g["acc"][targets]
    p99, pmax = per_particle(acc, ref["acc"])
    say(label, " ".join(f"{k}={v:.2e}" for k, v in errs.items()),
        f"acc per-particle p99={p99:.2e} max={pmax:.2e}")
    for k, e in errs.items():
        assert e <= tol, (label, k, e)
    assert p99 <= TOL_P99[precision], (label, "acc p99", p99)
    nn = g["nnb"] if targets is None else g["nnb"][targets]
    assert np.array_equal(nn.astype(np.int64), ref["nnb"])


# ---------------------------------------------------------------------------
# binning and neighbours: bit-exact
# ---------------------------------------------------------------------------

def hard_state(dim, seed):
    p, _, dp = None, None, None
    n_side = 16
    dp = 1.0 / n_side
    p = WL.base_params(dim, (1.0,) * dim, dp, (1.0, 1.0), (0.0, 0.0), 0.0, 1.0)
    ok, nc = O.grid(p)
    rng = np.random.default_rng(seed)
    pts = WL.lattice(dim, (n_side,) * dim, dp)
    pts = pts + rng.uniform(-0.3 * dp, 0.3 * dp, pts.shape)
    faces = np.array([[k / nc[0]] + [0.5 + 0.01 * k] * (dim - 1) for k in range(nc[0])])
    pos = O.wrap(p, np.vstack([pts, faces]))
    phase = (rng.uniform(size=pos.shape[0]) < 0.3).astype(np.int32)
    return p, pos, phase


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_binning_bit_exact(dim, precision):
    p, pos, phase = hard_state(dim, 4)
    say(f"binning dim={dim} precision={precision} n={len(pos)}")
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, np.zeros_like(pos), phase)
    key, rank = s.binning()
    kref = O.cell_keys(p, pos)
    perm, _ = O.bin_particles(p, kref, pos)
    rref = np.empty_like(perm)
    rref[perm] = np.arange(len(perm))
    assert np.array_equal(key, kref)
    assert np.array_equal(rank, rref)
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_neighbour_sets_equal_brute_force(dim, precision):
    p, pos, phase = hard_state(dim, 5)
    say(f"neighbours dim={dim} precision={precision} n={len(pos)}")
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, np.zeros_like(pos), phase)
    start, idx = s.neighbours()
    bs, bi = O.neighbours_brute(p, pos, cap_per=400)
    assert np.array_equal(start, bs)
    for i in range(len(pos)):
        assert np.array_equal(np.sort(idx[start[i]:start[i + 1]]), bi[bs[i]:bs[i + 1]])
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_neighbour_sets_on_large_compressed_lattices(dim, precision):
    """Many blocks whose stencil rows do not wrap, where the rows' first and
    last cells are cut to each particle's reach in x: a jittered lattice
    whose density varies by +-25 % along x and y (a periodic warp), against
    the oracle's cell search (itself pinned to brute force)."""
    n_side = 160 if dim == 2 else 36
    dp = 1.0 / n_side
    p = WL.base_params(dim, (1.0,) * dim, dp, (1.0, 1.0), (0.0, 0.0), 0.0, 1.0)
    rng = np.random.default_rng(11)
    pos = WL.lattice(dim, (n_side,) * dim, dp)
    pos = pos + rng.uniform(-0.3 * dp, 0.3 * dp, pos.shape)
    for a in range(2):
        pos[:, a] = pos[:, a] + 0.25 / (2 * np.pi) * np.sin(2 * np.pi * pos[:, a])
    pos = O.wrap(p, pos)
    phase = (rng.uniform(size=len(pos)) < 0.5).astype(np.int32)
    say(f"neighbours, warped lattice dim={dim} precision={precision} n={len(pos)}")
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, np.zeros_like(pos), phase)
    start, idx = s.neighbours(cap_per=300)
    rs, ri = O.neighbours_cells(p, pos, cap_per=300)
    assert np.array_equal(start, rs)
    owner = np.repeat(np.arange(len(pos)), np.diff(start))
    got = idx[:start[-1]][np.lexsort((idx[:start[-1]], owner))]
    assert np.array_equal(got, ri[:rs[-1]])  # the oracle's lists ascend in j
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("with_lattice", [False, True])
def test_neighbour_predicate_at_oblique_cut_off_pairs(dim, with_lattice):
    """Pairs at (2h)^2 where a fused multiply-add would decide otherwise than
    the plain sum, alone (blocks over many cell rows: the exact test of every
    candidate) and inside a lattice (the FP32 test with the exact test of the
    near-cut-off band): the GPU lists equal the oracle's brute force."""
    import cutoff_pairs as CP
    dp, pos, pp = CP.state(dim, 16, with_lattice, 3)
    p = WL.base_params(dim, (1.0,) * dim, dp, (1.0, 1.0), (0.0, 0.0), 0.0, 1.0)
    rng = np.random.default_rng(4)
    phase = (rng.uniform(size=len(pos)) < 0.3).astype(np.int32)
    say(f"cut-off pairs dim={dim} lattice={with_lattice} n={len(pos)}")
    s = rsph.System(p)
    s.set_particles(pos, np.zeros_like(pos), phase)
    start, idx = s.neighbours()
    bs, bi = O.neighbours_brute(p, pos, cap_per=400)
    assert np.array_equal(start, bs)
    for i in range(len(pos)):
        assert np.array_equal(np.sort(idx[start[i]:start[i + 1]]), bi[bs[i]:bs[i + 1]])
    s.close()


# ---------------------------------------------------------------------------
# single evaluations
# ---------------------------------------------------------------------------

CASES = {
    "droplet2d_ratio1000": lambda: WL.static_droplet_2d(n_side=50, R=0.2, seed=0),
    "droplet2d_ratio1": lambda: WL.static_droplet_2d(n_side=40, R=0.2, seed=2,
                                                      rho=(1.0, 1.0), eta=(0.05, 0.05)),
    "droplet3d_ratio1000": lambda: WL.static_droplet_3d(n_side=20, R=0.3, seed=0),
    "ellipse2d_ratio10": lambda: WL.oscillating_ellipse_2d(3000, 1.4, 10.0, 1.5, seed=3),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_eval_rates_parity(case, precision):
    w = CASES[case]()
    p, pos, vel, rho, mass, phase = perturbed_state(w)
    say(f"eval {case} precision={precision} n={len(pos)}")
    g = gpu_rates(p, pos, vel, rho, mass, phase, precision)
    ref = O.eval_rates(p, pos, vel, rho, mass, phase)
    compare_rates(g, ref, precision, f"{case}/p{precision}")


@pytest.mark.parametrize("flags", [rsph.NO_PENALTY, rsph.GBAR_OWN_PHASE_AVERAGE, rsph.PENALTY_R3,
                                   rsph.NO_SURFACE])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_eval_rates_parity_method_switches(flags, dim, precision):
    if dim == 2:
        w = WL.static_droplet_2d(n_side=40, R=0.2, seed=1)
    else:
        w = WL.static_droplet_3d(n_side=16, R=0.3, seed=1)
    p, pos, vel, rho, mass, phase = perturbed_state(w)
    p["flags"] = flags
    p["oracle_flags"] = flags
    say(f"eval switches flags={flags} dim={dim} precision={precision}")
    g = gpu_rates(p, pos, vel, rho, mass, phase, precision)
    ref = O.eval_rates(p, pos, vel, rho, mass, phase)
    compare_rates(g, ref, precision, f"flags{flags}/d{dim}/p{precision}")


@pytest.mark.parametrize("precision", [0, 1])
def test_momentum_conservation_on_gpu(precision):
    w = WL.static_droplet_3d(n_side=20, R=0.3, seed=4)
    p, pos, vel, rho, mass, phase = perturbed_state(w)
    s = rsph.System(p, precision=precision)
    s.set_particles(pos, vel, phase, mass=mass, rho=rho)
    s.eval_rates()
    tol = 1e-12 if precision == 0 else 1e-6
    for k in ["acc_p", "acc_s", "acc_v"]:
        f = mass[:, None] * s.read(k)
        tot = np.array([math.fsum(f[:, a]) for a in range(3)])
        scale = np.abs(f).sum()
        say(f"momentum p{precision} {k} {np.abs(tot).max() / scale:.2e}")
        assert np.abs(tot).max() <= tol * scale
    s.close()


def test_single_particle_and_single_phase_edge_cases():
    # one particle: no neighbours, zero rates except gravity
    p = WL.base_params(2, (1.0, 1.0), 0.05, (1.0, 1.0), (0.01, 0.01), 1.0, 1.0,
                       gravity=[0.0, -1.0, 0.0])
    s = rsph.System(p)
    s.set_particles(np.array([[0.5, 0.5]]), np.array([[0.1, 0.0]]), np.array([0], np.int32))
    s.eval_rates()
    assert np.allclose(s.read("acc"), [[0.0, -1.0]])
    assert s.read("nnb")[0] == 0
    s.step(2)
    o = s.observables()
    assert o["n_outer"] == 2 and o["n_sub"] >= 2
    s.close()
    # a single fluid: the colour gradient and surface terms vanish
    w = WL.static_droplet_2d(n_side=30, seed=5)
    p, pos, vel, rho, mass, phase = perturbed_state(w)
    phase = np.zeros_like(phase)
    g = gpu_rates(p, pos, vel, rho, mass, phase, 0)
    assert np.abs(g["gradC"]).max() == 0.0 and np.abs(g["acc_s"]).max() == 0.0


# ---------------------------------------------------------------------------
# trajectories
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_side", [50, 260])
def test_fp64_trajectory_matches_oracle(n_side):
    """4 advection steps of the static droplet.  At 2,500 particles the
    continuity pass ends each substep; at 67,600 (more than 1,024 force-pass
    blocks) a pass of its own does."""
    w = WL.static_droplet_2d(n_side=n_side, R=0.2, seed=0)
    p = w["params"]
    say(f"trajectory static droplet 2D n={len(w['pos'])}, 4 advection steps")
    st = O.State(p, w["pos"], w["vel"], w["phase"])
    st.step(4)
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(4)
    o = s.observables()
    ref = st.observables()
    assert o["n_outer"] == 4 and o["n_sub"] == ref["n_sub"]
    assert o["t"] == pytest.approx(ref["t"], rel=1e-12)
    ev = normwise(s.read("vel"), st.vel)
    er = normwise(s.read("rho") - np.asarray(p["rho0"])[w["phase"]],
                  st.rho - np.asarray(p["rho0"])[w["phase"]])
    pos = s.read("pos")
    dpos = pos - O.wrap(p, st.pos)
    dpos -= np.round(dpos)
    say(f"trajectory vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
    assert ev < 1e-9 and er < 1e-9 and np.abs(dpos).max() < 1e-12
    assert o["kinetic"] == pytest.approx(ref["kinetic"], rel=1e-9)
    s.close()


@pytest.mark.parametrize("case", ["no_shift", "no_density_summation", "no_penalty", "gravity"])
def test_fp64_trajectory_method_switches(case):
    """3 advection steps of the 2D static droplet under each switch that acts
    on the stepping (position shift, density summation, penalty) and with
    gravity, against the oracle."""
    w = WL.static_droplet_2d(n_side=40, R=0.2, seed=2)
    p = dict(w["params"])
    flags = {"no_shift": rsph.NO_SHIFT, "no_density_summation": rsph.NO_DENSITY_SUMMATION,
             "no_penalty": rsph.NO_PENALTY, "gravity": 0}[case]
    p["flags"] = flags
    p["oracle_flags"] = flags
    if case == "gravity":
        p["gravity"] = [0.0, -0.5, 0.0]
    say(f"trajectory switch {case}")
    st = O.State(p, w["pos"], w["vel"], w["phase"])
    st.step(3)
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(3)
    o = s.observables()
    ref = st.observables()
    assert o["n_outer"] == 3 and o["n_sub"] == ref["n_sub"]
    ev = normwise(s.read("vel"), st.vel)
    er = normwise(s.read("rho") - np.asarray(p["rho0"])[w["phase"]],
                  st.rho - np.asarray(p["rho0"])[w["phase"]])
    dpos = s.read("pos") - O.wrap(p, st.pos)
    dpos -= np.round(dpos)
    say(f"switch {case}: vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
    assert ev < 1e-9 and er < 1e-9 and np.abs(dpos).max() < 1e-12
    s.close()


def test_fp64_trajectory_large_pool_matches_oracle():
    """2 advection steps of a 2D static droplet of 1,048,576 particles in the
    FP64 form against the oracle: above a million slots the substep passes
    check the system's state before any slot load, and a separate pass ends
    each substep."""
    w = WL.static_droplet_2d(n_side=1024, R=0.2, seed=5)
    p = w["params"]
    say(f"trajectory static droplet 2D n={len(w['pos'])}, 2 advection steps")
    st = O.State(p, w["pos"], w["vel"], w["phase"])
    st.step(2)
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(2)
    o = s.observables()
    ref = st.observables()
    assert o["n_outer"] == 2 and o["n_sub"] == ref["n_sub"] and o["health"] == 0
    ev = normwise(s.read("vel"), st.vel)
    er = normwise(s.read("rho") - np.asarray(p["rho0"])[w["phase"]],
                  st.rho - np.asarray(p["rho0"])[w["phase"]])
    dpos = s.read("pos") - O.wrap(p, st.pos)
    dpos -= np.round(dpos)
    say(f"large pool trajectory vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
    assert ev < 1e-9 and er < 1e-9 and np.abs(dpos).max() < 1e-12
    s.close()


def test_fp64_trajectory_matches_oracle_3d_large():
    """2 advection steps (80 substeps) of a 3D static droplet of 74,088
    particles: past the fused-size limit, so a pass of its own ends each
    substep, in 3D."""
    w = WL.static_droplet_3d(n_side=42, R=0.25, seed=0)
    p = w["params"]
    say(f"trajectory static droplet 3D n={len(w['pos'])}, 2 advection steps")
    st = O.State(p, w["pos"], w["vel"], w["phase"])
    st.step(2)
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(2)
    o = s.observables()
    ref = st.observables()
    assert o["n_outer"] == 2 and o["n_sub"] == ref["n_sub"]
    assert o["t"] == pytest.approx(ref["t"], rel=1e-12)
    ev = normwise(s.read("vel"), st.vel)
    er = normwise(s.read("rho") - np.asarray(p["rho0"])[w["phase"]],
                  st.rho - np.asarray(p["rho0"])[w["phase"]])
    pos = s.read("pos")
    dpos = pos - O.wrap(p, st.pos)
    dpos -= np.round(dpos)
    say(f"trajectory 3D vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
    assert ev < 1e-9 and er < 1e-9 and np.abs(dpos).max() < 1e-12
    s.close()


# ---------------------------------------------------------------------------
# particle masses that differ within a fluid: the substep passes then gather
# each neighbour's volume (with one mass per fluid they recover it from the
# pressure the velocity record carries)
# ---------------------------------------------------------------------------

def varied_masses(p, phase, seed, spread=0.05):
    rng = np.random.default_rng(seed)
    d = p["dim"]
    base = np.asarray(list(p["rho0"]) + [1.0])[phase] / O.sigma0(d, p["dp"] * p.get("h_over_dp", 1.3), p["dp"])
    return base * (1.0 + spread * rng.uniform(-1.0, 1.0, size=len(phase)))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_eval_rates_parity_particle_masses(dim, precision):
    if dim == 2:
        w = WL.static_droplet_2d(n_side=40, R=0.2, seed=7)
    else:
        w = WL.static_droplet_3d(n_side=16, R=0.3, seed=7)
    p, pos, vel, rho, _, phase = perturbed_state(w, seed=8)
    mass = varied_masses(p, phase, seed=9)
    say(f"eval particle masses dim={dim} precision={precision}")
    g = gpu_rates(p, pos, vel, rho, mass, phase, precision)
    ref = O.eval_rates(p, pos, vel, rho, mass, phase)
    compare_rates(g, ref, precision, f"masses/d{dim}/p{precision}")


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_trajectory_particle_masses(precision, dim):
    """3 advection steps of a static droplet with particle masses spread by 5%
    within each fluid, against the oracle: the stepping path that gathers each
    neighbour's volume (in 3D the one-mass-per-fluid path is the default)."""
    if dim == 2:
        w = WL.static_droplet_2d(n_side=40, R=0.2, seed=3)
    else:
        w = WL.static_droplet_3d(n_side=16, R=0.3, seed=3)
    p = w["params"]
    mass = varied_masses(p, w["phase"], seed=4)
    say(f"trajectory particle masses dim={dim} precision={precision}")
    st = O.State(p, w["pos"], w["vel"], w["phase"], mass=mass)
    st.step(3)
    s = rsph.System(p, precision=precision)
    s.set_particles(w["pos"], w["vel"], w["phase"], mass=mass)
    s.step(3)
    o = s.observables()
    ref = st.observables()
    assert o["n_outer"] == 3 and o["health"] == 0
    # the mixed form's FP32 |v| maxima may shift a substep count by one
    assert abs(o["n_sub"] - ref["n_sub"]) <= (0 if precision == 0 else 3)
    ev = normwise(s.read("vel"), st.vel)
    er = normwise(s.read("rho") - np.asarray(p["rho0"])[w["phase"]],
                  st.rho - np.asarray(p["rho0"])[w["phase"]])
    dpos = s.read("pos") - O.wrap(p, st.pos)
    dpos -= np.round(dpos)
    say(f"particle masses p{precision}: vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
    if precision == 0:
        assert ev < 1e-9 and er < 1e-9 and np.abs(dpos).max() < 1e-12
    else:
        assert ev < 1e-4 and er < 1e-4 and np.abs(dpos).max() < 1e-4 * p["dp"]
    s.close()


def test_bitwise_determinism_and_resume():
    w = WL.static_droplet_2d(n_side=40, R=0.2, seed=6)
    p = w["params"]
    runs = []
    for _ in range(2):
        s = rsph.System(p, precision=1)
        s.set_particles(w["pos"], w["vel"], w["phase"])
        s.step(3)
        runs.append((s.read("pos"), s.read("vel"), s.read("rho")))
        s.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    # checkpoint after 1 step, resume for 2: bitwise equal to 3 straight steps
    s = rsph.System(p, precision=1)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    s.step(1)
    ck = {k: s.read(k) for k in ["pos", "vel", "rho", "drho", "mass"]}
    s.close()
    s = rsph.System(p, precision=1)
    s.set_particles(ck["pos"], ck["vel"], w["phase"], mass=ck["mass"], rho=ck["rho"])
    s.set_drho(ck["drho"])
    s.step(2)
    for a, k in zip(runs[0], ["pos", "vel", "rho"]):
        assert np.array_equal(a, s.read(k)), k
    s.close()


# ---------------------------------------------------------------------------
# full-size workloads, sampled outputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", [0, 1])
def test_static_droplet_3d_full_size_subset(precision):
    """262,144 particles; parity on the 16^3 lattice block straddling the
    interface (4,096 particles), the oracle evaluating that block only."""
    w = WL.static_droplet_3d(n_side=64, R=0.25, seed=0)
    p, pos, vel, rho, mass, phase = perturbed_state(w)
    say(f"3D full size precision={precision}")
    g = gpu_rates(p, pos, vel, rho, mass, phase, precision)
    targets = WL.subset_indices_3d(64, (40, 24, 24), (56, 40, 40))
    ref = O.eval_rates(p, pos, vel, rho, mass, phase, targets=targets)
    assert (phase[targets] == 0).sum() > 500
    compare_rates(g, ref, precision, f"c3subset/p{precision}", targets=targets)


def test_static_droplet_3d_mixed_against_fp64_along_the_run():
    """262,144 particles, at the states that the FP64 path reaches after 1, 10,
    100, 1,000 and 2,000 advection steps from the workload's start: one
    evaluation of every rate in the mixed form against the FP64 form at the
    same state, all particles, to the mixed form's tolerance.  The reference
    here is the FP64 GPU path, which the oracle pins at the start; no GPU state
    is handed to the oracle."""
    w = WL.static_droplet_3d(n_side=64, R=0.25, seed=0)
    p = w["params"]
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    done = 0
    for k in (1, 10, 100, 1000, 2000):
        s.step(k - done)
        done = k
        pos, vel, rho, mass = (s.read(f) for f in ("pos", "vel", "rho", "mass"))
        say(f"3D along the run: step {k}, max |v| {np.abs(vel).max():.3e}")
        g64 = gpu_rates(p, pos, vel, rho, mass, w["phase"], 0)
        g32 = gpu_rates(p, pos, vel, rho, mass, w["phase"], 1)
        errs = {f: normwise(g32[f], g64[f]) for f in FIELDS}
        say(f"step {k}", " ".join(f"{f}={e:.2e}" for f, e in errs.items()))
        for f, e in errs.items():
            assert e <= TOL[1], (k, f, e)
        assert np.array_equal(g32["nnb"], g64["nnb"])
    assert s.observables()["health"] == 0
    s.close()


def impact_input_sample(w, n, seed=9):
    """Particles chosen from the inputs alone: those whose initial position lies
    within 3h of the drop's or the pool's surface (n / 2 of them at random)
    and n / 2 drawn from all particles."""
    rng = np.random.default_rng(seed)
    h = w["params"]["dp"] * 1.3
    pos = w["pos"]
    near = np.abs(np.linalg.norm(pos - w["centre"], axis=1) - w["R"]) < 3 * h
    near |= np.abs(pos[:, 2] - w["pool_depth"]) < 3 * h
    near = rng.choice(np.where(near)[0], n // 2, replace=False)
    return np.unique(np.concatenate([near, rng.choice(len(pos), n // 2, replace=False)]))


@pytest.mark.parametrize("precision", [0, 1])
def test_droplet_impact_full_size_sampled(precision):
    """8,388,608 particles; parity on 2,000 particles chosen from the inputs,
    half of them within 3h of the drop's or the pool's surface."""
    w = WL.droplet_impact_3d()
    p, pos, vel, rho, mass, phase = perturbed_state(w, vscale=1.0)
    vel[w["vel"][:, 2] != 0, 2] -= 50.0
    say(f"impact full size n={len(pos)} precision={precision}")
    targets = impact_input_sample(w, 2000)
    g = gpu_rates(p, pos, vel, rho, mass, phase, precision)
    ref = O.eval_rates(p, pos, vel, rho, mass, phase, targets=targets)
    assert (np.linalg.norm(ref["gradC"], axis=1) > 0).sum() > 300
    compare_rates(g, ref, precision, f"impact/p{precision}", targets=targets)


def test_static_droplet_3d_subset_along_the_oracle_run():
    """262,144 particles, stepped by the oracle itself to advection steps 1 and
    10.  At each of those states both GPU forms evaluate every rate and are
    compared with the oracle on the 16^3 lattice block that straddles the
    interface (4,096 particles).  The FP64 GPU path also steps from the start
    and its block state is compared with the oracle's at both steps."""
    w = WL.static_droplet_3d(n_side=64, R=0.25, seed=0)
    p = w["params"]
    targets = WL.subset_indices_3d(64, (40, 24, 24), (56, 40, 40))
    st = O.State(p, w["pos"], w["vel"], w["phase"])
    s64 = rsph.System(p, precision=0)
    s64.set_particles(w["pos"], w["vel"], w["phase"])
    done = 0
    for k in (1, 10):
        say(f"3D oracle run: stepping to advection step {k}")
        st.step(k - done)
        s64.step(k - done)
        done = k
        pos = O.wrap(p, st.pos)
        ref = O.eval_rates(p, pos, st.vel, st.rho, st.mass, st.phase, targets=targets)
        for prec in (0, 1):
            g = gpu_rates(p, pos, st.vel, st.rho, st.mass, st.phase, prec)
            compare_rates(g, ref, prec, f"c3 oracle step {k} p{prec}", targets=targets)
        o = s64.observables()
        assert o["n_sub"] == st.clock.n_sub
        ev = normwise(s64.read("vel")[targets], st.vel[targets])
        er = normwise(s64.read("rho")[targets] - 1000.0 * (st.phase[targets] == 0) - (st.phase[targets] == 1),
                      st.rho[targets] - 1000.0 * (st.phase[targets] == 0) - (st.phase[targets] == 1))
        dpos = s64.read("pos")[targets] - pos[targets]
        dpos -= np.round(dpos)
        say(f"c3 FP64 trajectory step {k}: vel {ev:.2e} rho {er:.2e} pos {np.abs(dpos).max():.2e}")
        assert ev < 1e-8 and er < 1e-8 and np.abs(dpos).max() < 1e-12
    s64.close()


@pytest.mark.parametrize("case", ["droplet3d_ratio1000", "impact_box"])
def test_mixed_density_summation_is_near_fp64(case):
    """The mixed form's 3D density summation forms pair distances from 31-bit
    fixed-point offsets within each cell (within about 1e-9 h of the FP64
    distance), not from FP32 ones: its kernel sum sigma (section 2, the
    density summation) stays within 2e-8 of the oracle's, far inside the
    1e-5 of the FP32 pair loops, with walls (whose phase rides in the
    offsets' top bits) and without."""
    targets = None
    if case == "impact_box":
        w = WL.droplet_impact_wall_3d(n_per_unit=8)
        p = dict(w["params"])
        phase = w["phase"]
        rng = np.random.default_rng(4)
        n = len(phase)
        pos = O.wrap(p, w["pos"])
        vel = w["vel"].copy()
        rho0 = np.asarray(list(p["rho0"]) + [1.0])[phase]
        rho = rho0 * np.where(phase == 2, 1.0, 1.0 + 0.01 * rng.normal(size=n))
        mass = rho0 / O.sigma0(3, p["dp"] * 1.3, p["dp"])
        targets = np.unique(rng.choice(n, 4000, replace=False))
    else:
        p, pos, vel, rho, mass, phase = perturbed_state(CASES[case]())
    say(f"mixed density summation {case} n={len(pos)}")
    g = gpu_rates(p, pos, vel, rho, mass, phase, 1)
    ref = O.eval_rates(p, pos, vel, rho, mass, phase, targets=targets)
    sig = g["sigma"] if targets is None else g["sigma"][targets]
    err = normwise(sig, ref["sigma"])
    rel = np.abs(sig - ref["sigma"]) / np.abs(ref["sigma"])
    say(f"  sigma normwise {err:.2e}, per particle max {rel.max():.2e}")
    assert err <= 2e-8 and rel.max() <= 2e-8, (err, rel.max())
