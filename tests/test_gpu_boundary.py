"""Boundary rules that need a device: the sound-speed rule of section 2
(c0 = 0 in the parameters), and the count of advection steps that moved a
particle more than one cell."""
import sys

import numpy as np
import pytest

from paper_2503_16082_amd import workloads as WL

pytestmark = pytest.mark.gpu

rsph = pytest.importorskip("paper_2503_16082_amd.rsph")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def c0_of(s, rho, rho0):
    """c0 from the pressure of Eq. 3: p = c0^2 (rho - rho0)."""
    p = s.read("p")
    return float(np.sqrt(np.median(p / (rho - rho0))))


def test_sound_speed_rule_from_u_ref_and_the_initial_speed():
    """Section 2: c0 = 10 U_max.  With c0 = 0 the library takes U_max as the
    larger of u_ref and the largest initial speed."""
    w = WL.static_droplet_2d(n_side=30)
    p = dict(w["params"])
    p["c0"] = 0.0
    p["u_ref"] = 0.07
    n = len(w["pos"])
    rho0 = np.asarray(p["rho0"])[w["phase"]]
    rho = rho0 * (1.0 + 1e-3 * (1 + np.arange(n) % 7))
    s = rsph.System(p, precision=0)
    s.set_particles(w["pos"], w["vel"], w["phase"], rho=rho)
    assert c0_of(s, rho, rho0) == pytest.approx(0.7, rel=1e-9)
    vel = w["vel"].copy()
    vel[5] = (0.3, 0.4)  # |v| = 0.5 > u_ref
    s.set_particles(w["pos"], vel, w["phase"], rho=rho)
    assert c0_of(s, rho, rho0) == pytest.approx(5.0, rel=1e-9)
    s.step(1)
    assert s.observables()["health"] == 0
    s.close()


def test_sound_speed_rule_needs_a_speed():
    w = WL.static_droplet_2d(n_side=30)
    p = dict(w["params"])
    p["c0"] = 0.0
    p["u_ref"] = 0.0
    s = rsph.System(p, precision=0)
    with pytest.raises(rsph.RsphError) as e:
        s.set_particles(w["pos"], w["vel"], w["phase"])
    assert e.value.name == "EINVAL"
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_displacement_beyond_one_cell_is_counted(precision):
    """A perfect lattice under a strong uniform gravity: the viscous limit of
    Eq. 16 (0.1 rho0 h^2 / eta = 0.1) lets every particle fall g dt^2 / 2 = 0.5,
    three cells of edge 1/6, within one advection step; the next binning finds
    it and counts the step.  No pair force acts on a uniformly moving lattice,
    so the system stays healthy and keeps stepping."""
    n_side = 16
    dp = 1.0 / n_side
    h = 1.3 * dp
    eta = 0.1 * h * h / 0.1
    p = WL.base_params(2, (1.0, 1.0), dp, (1.0, 1.0), (eta, eta), 0.0, 1.0, gravity=[0.0, -100.0, 0.0])
    pts = WL.lattice(2, (n_side, n_side), dp)
    s = rsph.System(p, precision=precision)
    s.set_particles(pts, np.zeros_like(pts), np.zeros(len(pts), np.int32))
    s.step(1)
    o = s.observables()
    say(f"after one step: t={o['t']:.4f} dt_ad={o['dt_ad']:.4f} displaced={o['displaced_steps']}")
    assert o["health"] == 0 and o["dt_ad"] == pytest.approx(0.1, rel=1e-12)
    assert o["displaced_steps"] == 0
    s.step(1)
    o = s.observables()
    assert o["health"] == 0 and o["displaced_steps"] == 1
    # a slow lattice (no gravity) is never counted
    p["gravity"] = [0.0, 0.0, 0.0]
    q = rsph.System(p, precision=precision)
    q.set_particles(pts, np.full_like(pts, 1e-3), np.zeros(len(pts), np.int32))
    q.step(3)
    assert q.observables()["displaced_steps"] == 0
    s.close()
    q.close()
