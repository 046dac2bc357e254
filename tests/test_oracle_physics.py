"""The oracle against the paper's dynamic results (section 5.1), on the CPU.

* Ratio 1000, V0 = 1 (Eq. 34 start): the mode-2 period of the drop is that of
  Eq. 35 within the paper's 5 %.
* Ratio 1, V0 = 10, eta = 0.05 at R/dp = 6, 12 and 24 (900, 3,600 and 14,400
  particles): the centre of mass of the drop's upper-right quarter follows one
  curve that converges with resolution (the paper's convergence figure for this
  case): the R/dp = 12 curve lies closer to the R/dp = 24 curve than the
  R/dp = 6 curve does, and within 0.25 dp of it.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_16082_amd import workloads as WL

from physics_util import measured_period, theory_period, trace, upper_right_quarter_centre


def test_oracle_oscillating_drop_period_matches_eq35():
    gamma = 1.0
    w = WL.oscillating_drop_2d(n_side=60, ratio=1000.0, V0=1.0, gamma=gamma)
    tau = theory_period(w["R"], w["params"]["rho0"][0], gamma)
    st = O.State(w["params"], O.wrap(w["params"], w["pos"]), w["vel"], w["phase"])
    ts, ds = trace(st.step, st.observables, 1.6 * tau)
    por = measured_period(ts, ds, tau)
    print(f"oracle period {por:.5f}, Eq. 35 {tau:.5f} ({100 * (por / tau - 1):+.2f} %)")
    assert abs(por / tau - 1.0) < 0.05


def quarter_centre_track(stepper, observe, positions, phase, t_end, every=10):
    """x of the upper-right quarter's centre of mass (relative to fluid k's
    centroid), sampled every `every` advection steps until t_end."""
    ts, xs = [], []
    while True:
        o = observe()
        ts.append(o["t"])
        xs.append(upper_right_quarter_centre(positions(), phase, o["centroid"])[0])
        if o["t"] >= t_end:
            return np.array(ts), np.array(xs)
        stepper(every)


def ratio1_drop(r_over_dp):
    return WL.oscillating_drop_2d(n_side=int(round(r_over_dp / 0.2)), ratio=1.0, V0=10.0, gamma=1.0)


def test_oracle_ratio1_drop_converges_with_resolution():
    t_end = 0.5
    tq = np.linspace(0.02, t_end, 25)
    curves = {}
    for r_dp in (6, 12, 24):
        w = ratio1_drop(r_dp)
        p = w["params"]
        st = O.State(p, O.wrap(p, w["pos"]), w["vel"], w["phase"])
        ts, xs = quarter_centre_track(st.step, st.observables, lambda: st.pos, st.phase, t_end)
        curves[r_dp] = np.interp(tq, ts, xs)
    e6 = np.abs(curves[6] - curves[24]).max()
    e12 = np.abs(curves[12] - curves[24]).max()
    print(f"max |x_6 - x_24| = {e6:.2e}, max |x_12 - x_24| = {e12:.2e}")
    assert e12 < e6
    assert e12 < 0.25 * 0.2 / 24
    # the drop stretches along x first (V0 > 0), then recoils
    x = curves[24]
    assert x.argmax() < x.argmin()
    assert x.max() - x.min() > 0.015
