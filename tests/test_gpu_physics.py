"""Physics validation: the oscillating drop of section 5.1.

A disc of fluid k (R = 0.2, density ratio 1000, viscosity ratio 100) starts
with the divergence-free velocity field of Eq. 34 (V0 = 1).  Small-deformation
theory gives the mode-2 capillary period of Eq. 35, tau = 2 pi sqrt(R^3 rho_k /
(6 gamma)).  The measured period is twice the mean spacing of the zero
crossings of D = (I_xx - I_yy) / (I_xx + I_yy), the normalised second moment of
fluid k about its centroid; crossings before 0.2 tau (the start-up) are
skipped.  The paper reports agreement within 5 %; the mixed form must give the
FP64 form's period within 1 %, and the FP64 form the oracle's.
"""
import math
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


def deformation(o):
    m = o["moment2"]
    return (m[0, 0] - m[1, 1]) / (m[0, 0] + m[1, 1])


def theory_period(R, rho_k, gamma):
    return 2.0 * math.pi * math.sqrt(R ** 3 * rho_k / (6.0 * gamma))


def measured_period(ts, ds, tau):
    cross = []
    for k in range(1, len(ts)):
        if ts[k] < 0.2 * tau:
            continue
        if (ds[k - 1] > 0) != (ds[k] > 0):
            f = ds[k - 1] / (ds[k - 1] - ds[k])
            cross.append(ts[k - 1] + f * (ts[k] - ts[k - 1]))
    assert len(cross) >= 2, cross
    return 2.0 * (cross[-1] - cross[0]) / (len(cross) - 1)


def trace(stepper, observe, t_end, every=5):
    ts, ds = [0.0], [deformation(observe())]
    while ts[-1] < t_end:
        stepper(every)
        o = observe()
        assert o.get("health", 0) == 0
        ts.append(o["t"])
        ds.append(deformation(o))
    return ts, ds


def gpu_period(w, precision, tau):
    s = rsph.System(w["params"], precision=precision)
    s.set_particles(w["pos"], w["vel"], w["phase"])
    ts, ds = trace(s.step, s.observables, 1.6 * tau)
    s.close()
    return measured_period(ts, ds, tau)


@pytest.mark.parametrize("gamma", [0.5, 1.0, 2.0])
def test_oscillating_drop_period(gamma):
    w = WL.oscillating_drop_2d(n_side=60, ratio=1000.0, V0=1.0, gamma=gamma)
    tau = theory_period(w["R"], w["params"]["rho0"][0], gamma)
    p64 = gpu_period(w, rsph.FP64, tau)
    pmx = gpu_period(w, rsph.MIXED, tau)
    say(f"gamma={gamma} tau(Eq. 35)={tau:.5f} fp64={p64:.5f} ({100 * (p64 / tau - 1):+.2f}%) "
        f"mixed={pmx:.5f} ({100 * (pmx / tau - 1):+.2f}%)")
    assert abs(p64 / tau - 1.0) < 0.05
    assert abs(pmx / tau - 1.0) < 0.05
    assert abs(pmx / p64 - 1.0) < 0.01


def test_oscillating_drop_period_gpu_matches_oracle():
    gamma = 1.0
    w = WL.oscillating_drop_2d(n_side=60, ratio=1000.0, V0=1.0, gamma=gamma)
    tau = theory_period(w["R"], w["params"]["rho0"][0], gamma)
    p64 = gpu_period(w, rsph.FP64, tau)
    st = O.State(w["params"], O.wrap(w["params"], w["pos"]), w["vel"], w["phase"])
    ts, ds = trace(st.step, st.observables, 1.6 * tau)
    por = measured_period(ts, ds, tau)
    say(f"oracle period {por:.5f} ({100 * (por / tau - 1):+.2f}%), GPU FP64 {p64:.5f}")
    assert abs(por / tau - 1.0) < 0.05
    assert abs(p64 / por - 1.0) < 0.01
