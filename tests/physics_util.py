"""Shared observables of the physics checks: the mode-2 deformation of fluid k
and the oscillation period from its zero crossings (section 5.1, Eq. 35)."""
import math

import numpy as np


def deformation(o):
    """D = (I_xx - I_yy) / (I_xx + I_yy) of fluid k's second moment."""
    m = o["moment2"]
    return (m[0, 0] - m[1, 1]) / (m[0, 0] + m[1, 1])


def theory_period(R, rho_k, gamma):
    """Eq. 35: tau = 2 pi sqrt(R^3 rho_k / (6 gamma))."""
    return 2.0 * math.pi * math.sqrt(R ** 3 * rho_k / (6.0 * gamma))


def measured_period(ts, ds, tau):
    """Twice the mean spacing of the zero crossings of D, skipping the start-up
    before 0.2 tau."""
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
    """(t, D) sampled every `every` advection steps until t_end."""
    ts, ds = [0.0], [deformation(observe())]
    while ts[-1] < t_end:
        stepper(every)
        o = observe()
        assert o.get("health", 0) == 0
        ts.append(o["t"])
        ds.append(deformation(o))
    return ts, ds


def upper_right_quarter_centre(pos, phase, centre):
    """Centre of mass (equal masses within fluid k) of the fluid-k particles in
    the drop's upper-right quarter, relative to the drop's centre."""
    d = pos - np.asarray(centre)
    sel = (phase == 0) & (d[:, 0] > 0) & (d[:, 1] > 0)
    return d[sel].mean(axis=0)
