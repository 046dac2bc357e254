"""Hand-solved pins of the oracle's individual terms, its integrator and its
observables.

Each expected value is worked out here for a configuration small or regular
enough to be solved by hand from the paper's equations (two or three
particles, a perfect lattice under uniform gravity, a symmetric constructed
state), so that a swapped average, a dropped weight, a transposed projection or
a misplaced half step in the oracle fails at least one of them.  The kernel
derivative used in the hand solutions is the oracle's, which is pinned on its
own against the textbook Wendland function.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_16082_amd import workloads as WL


DP = 1.0 / 30


def _params(rho0, eta=(0.0, 0.0), gamma=0.0, c0=10.0, dim=2, **kw):
    return WL.base_params(dim, (1.0,) * dim, DP, rho0, eta, gamma, c0, **kw)


def _dW(dim, r):
    return O.dW(dim, 1.3 * DP, r)


# --------------------------------------------------------------------------
# Eqs. 8-12 at unequal densities (density ratio 1000)
# --------------------------------------------------------------------------

def _pair_ratio_1000(u):
    """Particle 0 of fluid k (rho0 1000) at the centre, particle 1 of fluid l
    (rho0 1) at +r along x; velocities +u and -u along x (approaching for
    u > 0); pressures p0 = c0^2 (rho0 - 1000) = 200 and p1 = 50."""
    c0 = 10.0
    p = _params((1000.0, 1.0), c0=c0)
    r = 1.2 * DP
    pos = np.array([[0.5, 0.5], [0.5 + r, 0.5]])
    vel = np.array([[u, 0.0], [-u, 0.0]])
    rho = np.array([1000.0 + 200.0 / c0 ** 2, 1.0 + 50.0 / c0 ** 2])
    mass = np.array([1000.0, 1.0]) * DP * DP
    phase = np.array([0, 1], np.int32)
    return p, pos, vel, rho, mass, phase, r, c0


def test_pressure_average_is_density_weighted_at_ratio_1000():
    """At rest (beta = 0): P* = (rho_0 p_1 + rho_1 p_0) / (rho_0 + rho_1)
    (Eq. 12), a^p_0 = -(2/rho_0) P* dW e_01 V_1 (Eq. 7) with e_01 = -x.  The
    other weighting, (rho_0 p_0 + rho_1 p_1)/(rho_0 + rho_1), is ~4x larger."""
    p, pos, vel, rho, mass, phase, r, c0 = _pair_ratio_1000(0.0)
    out = O.eval_rates(p, pos, vel, rho, mass, phase)
    p0, p1 = 200.0, 50.0
    pstar = (rho[0] * p1 + rho[1] * p0) / (rho[0] + rho[1])
    dW = _dW(2, r)
    V0, V1 = mass / rho
    assert out["acc_p"][0, 0] == pytest.approx(-2.0 / rho[0] * pstar * dW * (-1.0) * V1, rel=1e-12)
    assert out["acc_p"][1, 0] == pytest.approx(-2.0 / rho[1] * pstar * dW * (+1.0) * V0, rel=1e-12)
    assert np.abs(out["acc_p"][:, 1]).max() == 0.0
    wrong = (rho[0] * p0 + rho[1] * p1) / (rho[0] + rho[1])
    assert abs(wrong / pstar - 1.0) > 1.0


def test_riemann_dissipation_and_star_velocity_at_ratio_1000():
    """Approaching pair, u = 0.2: U_L - U_R = 2u, beta = min(3 * 2u / c0, 1)
    (Eq. 11 with the pressures read as densities), P* = pbar + beta Z_L Z_R
    (U_L - U_R) / (Z_L + Z_R) (Eq. 8), Z = rho c0; continuity with the star
    velocity U* = (Z_L U_L + Z_R U_R + p_L - p_R) / (Z_L + Z_R) (Eq. 9) and
    D rho_i = 2 rho_i (v_i . e_ij + U*) dW V_j (Eq. 6 on the i->j axis)."""
    u = 0.2
    p, pos, vel, rho, mass, phase, r, c0 = _pair_ratio_1000(u)
    out = O.eval_rates(p, pos, vel, rho, mass, phase)
    pr = np.array([200.0, 50.0])
    Z = rho * c0
    dW = _dW(2, r)
    V = mass / rho
    beta = min(6.0 * u / c0, 1.0)
    pbar = (rho[0] * pr[1] + rho[1] * pr[0]) / (rho[0] + rho[1])
    pstar = pbar + beta * Z[0] * Z[1] * 2.0 * u / (Z[0] + Z[1])
    assert out["acc_p"][0, 0] == pytest.approx(-2.0 / rho[0] * pstar * dW * (-1.0) * V[1], rel=1e-12)
    assert out["acc_p"][1, 0] == pytest.approx(-2.0 / rho[1] * pstar * dW * (+1.0) * V[0], rel=1e-12)
    # particle 0: e_01 = -x, U_L = -v_0 . e_01 = u, U_R = -v_1 . e_01 = -u, v_0 . e_01 = -u
    ustar0 = (Z[0] * u + Z[1] * (-u) + pr[0] - pr[1]) / (Z[0] + Z[1])
    assert out["drho"][0] == pytest.approx(2 * rho[0] * (-u + ustar0) * dW * V[1], rel=1e-12)
    # particle 1: e_10 = +x, U_L = -v_1 . e_10 = u, U_R = -v_0 . e_10 = -u, v_1 . e_10 = -u
    ustar1 = (Z[1] * u + Z[0] * (-u) + pr[1] - pr[0]) / (Z[0] + Z[1])
    assert out["drho"][1] == pytest.approx(2 * rho[1] * (-u + ustar1) * dW * V[0], rel=1e-12)


# --------------------------------------------------------------------------
# Eq. 13 with unequal viscosities
# --------------------------------------------------------------------------

def test_viscous_acceleration_uses_the_harmonic_mean():
    """a^v_0 = (2/rho_0) [2 eta_0 eta_1 / (eta_0 + eta_1)] (v_0 - v_1) dW / r V_1;
    at eta = (0.3, 0.01) the harmonic mean is 0.0194, the arithmetic 0.155."""
    p = _params((2.0, 1.0), eta=(0.3, 0.01))
    r = 1.7 * DP
    pos = np.array([[0.5, 0.5], [0.5 + 0.6 * r, 0.5 + 0.8 * r]])
    vel = np.array([[0.2, 0.1], [-0.1, 0.3]])
    rho = np.array([2.1, 0.9])
    mass = np.array([2.0, 1.0]) * DP * DP
    phase = np.array([0, 1], np.int32)
    out = O.eval_rates(p, pos, vel, rho, mass, phase)
    eta_bar = 2 * 0.3 * 0.01 / 0.31
    dW = _dW(2, r)
    V = mass / rho
    expect0 = 2.0 / rho[0] * eta_bar * (vel[0] - vel[1]) * dW / r * V[1]
    expect1 = 2.0 / rho[1] * eta_bar * (vel[1] - vel[0]) * dW / r * V[0]
    assert np.allclose(out["acc_v"][0], expect0, rtol=1e-12, atol=0)
    assert np.allclose(out["acc_v"][1], expect1, rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# Eq. 24 surface stress: Pi n = 0 and tr Pi = (d - 1) gamma |grad C|
# --------------------------------------------------------------------------

def _stress_configuration(dim):
    """Particle 0 (fluid k) at the centre; particle 1 (fluid l) at -a along y,
    the only cross-phase neighbour of particle 0; particles 2 (and 3 in 3D) of
    fluid k at +b along x (and z), out of reach of particle 1 and of each other
    (a = b = 2 dp, sqrt(a^2 + b^2) = 2.83 dp > 2h = 2.6 dp)."""
    a = b = 2.0 * DP
    c = np.full(dim, 0.5)
    pts = [c.copy(), c.copy(), c.copy()]
    pts[1][1] -= a
    pts[2][0] += b
    if dim == 3:
        pts.append(c.copy())
        pts[3][2] += b
    pos = np.array(pts)
    n = pos.shape[0]
    phase = np.zeros(n, np.int32)
    phase[1] = 1
    return pos, phase, a, b


@pytest.mark.parametrize("dim", [2, 3])
def test_surface_stress_is_tangential_with_trace_d_minus_1(dim):
    """With the penalty off: grad C_0 = 2 phi_0 dW(a) V_1 e_01 (Eq. 22), so
    n_0 = -y and Pi_0 = gamma |grad C_0| (I - y y^T) (Eq. 24).  The normal pair
    (0, 1) carries no stress force (Pi e_01 = 0 for both particles), and each
    tangential same-phase neighbour k pulls particle 0 with (1/rho_0) Pi_0
    grad W_0k V_k (Eq. 26, Pi_k = 0 since k has no cross-phase neighbour): the
    same magnitude gamma |grad C_0| |dW(b)| V_k / rho_0 along x and (3D) z, which
    is the trace (d - 1) gamma |grad C_0| spread over the tangent plane."""
    pos, phase, a, b = _stress_configuration(dim)
    gamma = 1.7
    p = _params((10.0, 1.0), gamma=gamma, dim=dim, oracle_flags=O.NO_PENALTY)
    n = pos.shape[0]
    rho = np.array([10.0, 1.0, 10.0, 10.0][:n]) * (1.0 + 0.01 * np.arange(n))
    mass = np.array([10.0, 1.0, 10.0, 10.0][:n]) * DP ** dim
    out = O.eval_rates(p, pos, np.zeros_like(pos), rho, mass, phase)
    V = mass / rho
    phi0 = 10.0 / 11.0
    g0 = 2 * phi0 * abs(_dW(dim, a)) * V[1]
    assert np.linalg.norm(out["gradC"][0]) == pytest.approx(g0, rel=1e-13)
    assert out["gradC"][0][1] < 0
    assert np.abs(out["gradC"][2:]).max() == 0.0
    pull = gamma * g0 * abs(_dW(dim, b)) / rho[0]
    expect = np.zeros(dim)
    expect[0] = pull * V[2]
    if dim == 3:
        expect[2] = pull * V[3]
    assert np.allclose(out["acc_s"][0], expect, rtol=1e-12, atol=1e-12 * pull)
    # particle 1 feels nothing from the normal pair; particle 2 the reaction
    assert np.abs(out["acc_s"][1]).max() <= 1e-12 * pull
    assert out["acc_s"][2][0] == pytest.approx(-gamma * g0 * abs(_dW(dim, b)) * V[0] / rho[2], rel=1e-12)


def test_cross_phase_stress_weights_the_neighbours_stress_by_own_phi():
    """Across phases Eq. 33 weights the neighbour's stress by 2 phi_i (i's own
    share).  Particle 0 (fluid k, rho0 10) at the centre, particle 1 (fluid l,
    rho0 1) 1.5 dp below it, and particle 3 (fluid k) 2.2 dp to the right of 1,
    out of reach of 0.  grad C_0 lies along y, so Pi_0 e_01 = 0; particle 1 has
    two cross-phase neighbours, so Pi_1 e_01 is not zero and the surface
    acceleration of 0 (penalty off) is (1/rho_0) 2 phi_0 Pi_1 dW(a) e_01 V_1,
    with 2 phi_0 = 20/11 where the swapped weight would give 2/11."""
    gamma = 1.1
    a, b = 1.5 * DP, 2.2 * DP
    pos = np.array([[0.5, 0.5], [0.5, 0.5 - a], [0.5 + b, 0.5 - a]])
    phase = np.array([0, 1, 0], np.int32)
    rho = np.array([10.0 * 1.01, 1.02, 10.0 * 0.99])
    mass = np.array([10.0, 1.0, 10.0]) * DP * DP
    V = mass / rho
    p = _params((10.0, 1.0), gamma=gamma, oracle_flags=O.NO_PENALTY)
    out = O.eval_rates(p, pos, np.zeros_like(pos), rho, mass, phase)
    phi0, phi1 = 10.0 / 11.0, 1.0 / 11.0
    # Eq. 22 for particle 1: its neighbours of the other fluid are 0 (e_10 = -y)
    # and the third particle (e_13 = -x)
    g1 = 2 * phi1 * (_dW(2, a) * V[0] * np.array([0.0, -1.0]) + _dW(2, b) * V[2] * np.array([-1.0, 0.0]))
    assert out["gradC"][1] == pytest.approx(g1, rel=1e-13)
    gn = np.linalg.norm(g1)
    nh = g1 / gn
    Pi1 = gamma * gn * (np.eye(2) - np.outer(nh, nh))
    expect = 2 * phi0 * (Pi1 @ np.array([0.0, 1.0])) * _dW(2, a) * V[1] / rho[0]
    assert out["acc_s"][0] == pytest.approx(expect, rel=1e-12, abs=1e-14 * np.abs(expect).max())


# --------------------------------------------------------------------------
# Penalty (Eqs. 25-33): projections N-bar across and T-bar within a phase
# --------------------------------------------------------------------------

def test_penalty_on_a_normal_cross_phase_pair():
    """Two particles along y (0 of fluid k above 1 of fluid l), density ratio
    10, xi = 2, gamma = 1.3.  grad C_0 = 2 phi_0 dW V_1 y, grad C_1 = -2 phi_1 dW
    V_0 y.  Along the normal every reading of Eq. 30 gives Chat grad W =
    dW (1 - |gbar| r) e_01 with gbar the mean gradient of Eq. 27; N-bar = y y^T
    keeps it and the stress terms vanish, so a^s_0 = -(4 phi_0 phi_1 xi gamma /
    (rho_0 r)) dW (1 - |gbar| r) V_1 y (Eq. 33).  The one-field mean (default)
    has |gbar| = |dW| (phi_0 V_1 + phi_1 V_0), the printed own-phase average
    |dW| |phi_0 V_1 - phi_1 V_0|."""
    gamma, xi = 1.3, 2.0
    r = 1.4 * DP
    pos = np.array([[0.5, 0.5 + r], [0.5, 0.5]])
    rho = np.array([10.0 * 1.02, 0.97])
    mass = np.array([10.0, 1.0]) * DP * DP
    phase = np.array([0, 1], np.int32)
    V = mass / rho
    phi0, phi1 = 10.0 / 11.0, 1.0 / 11.0
    dW = _dW(2, r)
    for flags, gbar in ((0, abs(dW) * (phi0 * V[1] + phi1 * V[0])),
                        (O.GBAR_OWN_PHASE_AVERAGE, abs(dW) * abs(phi0 * V[1] - phi1 * V[0])),
                        (O.PENALTY_R3, abs(dW) * (phi0 * V[1] + phi1 * V[0]))):
        p = _params((10.0, 1.0), gamma=gamma, xi=xi, oracle_flags=flags)
        out = O.eval_rates(p, pos, np.zeros_like(pos), rho, mass, phase)
        k = 4 * phi0 * phi1 * xi * gamma / r * dW * (1.0 - gbar * r)
        assert out["acc_s"][0] == pytest.approx([0.0, -k * V[1] / rho[0]], rel=1e-12, abs=1e-14 * abs(k))
        assert out["acc_s"][1] == pytest.approx([0.0, +k * V[0] / rho[1]], rel=1e-12, abs=1e-14 * abs(k))


def test_penalty_within_a_phase_is_projected_tangentially():
    """Particle 0 (fluid k) at the centre with particle 1 (fluid l) 1.5 dp
    below it and particle 2 (fluid k) at (2.4, 0.5) dp, out of reach of 1.
    grad C_2 = 0 so T_2 = I and T-bar = (T_0 + I)/2 = diag(1, 1/2); N_0 = y y^T.
    gbar_02 = grad C_0 / 2 = g y (g < 0), r_02 = (-2.4, -0.5) dp.
    Reading R1 (default): Chat grad W = -dW (gbar . r_02) gbar/|gbar|, along y,
    halved by T-bar.  Reading R3: dW [-(gbar . r)^2 / (|gbar| r)] e_02, whose
    x part T-bar keeps whole.  The normal pair (0, 1) adds its N-bar penalty and
    the tangential stress term of (0, 2) adds gamma |grad C_0| dW e_02,x V_2."""
    gamma, xi = 0.8, 3.0
    a = 1.5 * DP
    d02 = np.array([2.4, 0.5]) * DP
    pos = np.array([[0.5, 0.5], [0.5, 0.5 - a], [0.5 + d02[0], 0.5 + d02[1]]])
    phase = np.array([0, 1, 0], np.int32)
    rho = np.array([10.0 * 1.01, 0.99, 10.0 * 0.995])
    mass = np.array([10.0, 1.0, 10.0]) * DP * DP
    V = mass / rho
    phi0, phi1 = 10.0 / 11.0, 1.0 / 11.0
    dWa = _dW(2, a)
    r2 = float(np.linalg.norm(d02))
    dW2 = _dW(2, r2)
    e02 = -d02 / r2
    # colour gradients (Eq. 22)
    gC0 = 2 * phi0 * dWa * V[1]          # y component (negative)
    gC1 = -2 * phi1 * dWa * V[0]         # y component (positive)
    # (0, 1): normal cross-phase pair, one-field mean, N-bar = y y^T
    G = abs(0.5 * (gC0 - gC1))
    pen01 = -(4 * phi0 * phi1 * xi * gamma / a) * dWa * (1.0 - G * a) * V[1]
    # (0, 2): stress term, Pi_0 = gamma |gC0| x x^T, Pi_2 = 0
    st02 = gamma * abs(gC0) * dW2 * e02[0] * V[2]
    g = 0.5 * gC0
    gdotr = g * (-d02[1])
    for flags in (0, O.PENALTY_R3):
        p = _params((10.0, 1.0), gamma=gamma, xi=xi, oracle_flags=flags)
        out = O.eval_rates(p, pos, np.zeros_like(pos), rho, mass, phase)
        if flags == 0:
            # q = -dW (gbar . r) ghat with ghat = -y; T-bar y = y / 2
            q = np.array([0.0, -dW2 * gdotr * (-1.0)])
            tq = np.array([q[0], 0.5 * q[1]])
        else:
            s = -(gdotr ** 2) / (abs(g) * r2)
            q = dW2 * s * e02
            tq = np.array([q[0], 0.5 * q[1]])
        pen02 = xi * gamma / r2 * tq * V[2]
        expect = (np.array([st02, pen01]) + pen02) / rho[0]
        assert out["acc_s"][0] == pytest.approx(expect, rel=1e-11, abs=1e-13 * np.abs(expect).max())
    # the two readings differ in direction: R1 has no x penalty, R3 has one
    assert abs(dW2 * (-(gdotr ** 2) / (abs(g) * r2)) * e02[0]) > 1e-6 * abs(pen01)


# --------------------------------------------------------------------------
# The integrator (section 3.3) in closed form: a perfect lattice under gravity
# --------------------------------------------------------------------------

def test_lattice_under_gravity_follows_the_closed_form_trajectory():
    """Two fluids on a perfect periodic lattice (no surface tension) feel no
    pair force, so every particle moves as x0 + g t^2 / 2 with v = g t, which
    kick-drift-kick integrates exactly for any sequence of substeps.  Eq. 16 is
    viscosity-limited (0.1 rho0_l h^2 / eta_l = 0.66 < 0.1 h / |v|) and Eq. 17
    gives an acoustic step of about 0.29 of it, so every advection step takes
    four substeps, the last one clipped so that the clock lands on whole
    advection steps: t = n dt_ad."""
    n_side = 16
    dp = 1.0 / n_side
    h = 1.3 * dp
    dt_ad = 0.1 * 1.0 * h * h / 1e-3
    c0 = 0.6 * h / (0.29 * dt_ad)
    p = WL.base_params(2, (1.0, 1.0), dp, (1000.0, 1.0), (0.1, 1e-3), 0.0, c0,
                       gravity=[0.0, 1e-3, 0.0])
    pts = WL.lattice(2, (n_side, n_side), dp)
    phase = np.where(pts[:, 0] < 0.5, 0, 1).astype(np.int32)
    st = O.State(p, pts, np.zeros_like(pts), phase)
    steps = 5
    st.step(steps)
    o = st.observables()
    t = o["t"]
    assert o["dt_ad"] == pytest.approx(dt_ad, rel=1e-14)
    assert t == pytest.approx(steps * dt_ad, rel=1e-13)
    assert o["n_sub"] == 4 * steps
    assert 0 < o["dt_ac"] < 0.6 * h / c0
    g = 1e-3
    assert np.allclose(st.vel[:, 1], g * t, rtol=1e-11, atol=0)
    assert np.abs(st.vel[:, 0]).max() < 1e-9 * g * t
    dy = (st.pos[:, 1] - pts[:, 1] + 0.5) % 1.0 - 0.5
    assert np.allclose(dy, 0.5 * g * t * t, rtol=0, atol=1e-13)
    dx = (st.pos[:, 0] - pts[:, 0] + 0.5) % 1.0 - 0.5
    assert np.abs(dx).max() < 1e-13
    assert np.allclose(st.rho, np.asarray(p["rho0"])[phase], rtol=1e-13)


# --------------------------------------------------------------------------
# Observables on a constructed state
# --------------------------------------------------------------------------

def test_observables_of_a_constructed_state():
    """Fluid k: four particles at distance 0.01 from (0.5, 0.5) on the axes,
    four at 0.2 and two at 0.3 on the x axis, each of volume 0.01, so
    r_eq = sqrt(0.1 / pi) = 0.1784; fluid l: particles at 0.071, 0.12, 0.27 and
    0.4 from the centre.  h = 0.026: the inner mean takes fluid-k particles with
    |r - c| < r_eq - 3h = 0.1004 (the four near ones, not the fluid-l particle at
    0.071) and the outer mean fluid-l particles with |r - c| > r_eq + 3h = 0.2564
    (those at 0.27 and 0.4, not the fluid-k pair at 0.3)."""
    c0 = 2.0
    p = WL.base_params(2, (1.0, 1.0), 0.02, (1.0, 0.5), (0.0, 0.0), 0.0, c0)
    a, A, B = 0.01, 0.2, 0.3
    k_off = [(a, 0), (-a, 0), (0, a), (0, -a), (A, 0), (-A, 0), (0, A), (0, -A), (B, 0), (-B, 0)]
    l_off = [(0.05, 0.05), (0.12, 0.0), (0.27, 0.0), (0.0, -0.4)]
    pos = 0.5 + np.array(k_off + l_off, dtype=np.float64)
    nk = len(k_off)
    phase = np.array([0] * nk + [1] * len(l_off), np.int32)
    # fluid k at rho0 = 1 except the inner four, whose pressures c0^2 (rho - 1)
    # are 0.1, 0.2, 0.3, 0.4; masses m = 0.01 rho keep every volume at 0.01
    rho = np.ones(pos.shape[0])
    rho[:4] = 1.0 + np.array([0.1, 0.2, 0.3, 0.4]) / c0 ** 2
    rho[nk:] = 0.5 + np.array([0.04, 0.03, -0.02, 0.01]) / c0 ** 2
    mass = np.concatenate([0.01 * rho[:nk], np.full(len(l_off), 0.005)])
    vel = np.zeros_like(pos)
    vel[0] = (0.3, 0.0)
    vel[1] = (-0.3, 0.0)
    vel[nk + 1] = (0.0, 2.0)
    st = O.State(p, pos, vel, phase, mass=mass, rho=rho)
    o = st.observables()
    m = mass
    M = m[:nk].sum()
    assert o["momentum"] == pytest.approx([(m[0] - m[1]) * 0.3, 0.005 * 2.0], abs=1e-15)
    assert o["kinetic"] == pytest.approx(0.5 * ((m[0] + m[1]) * 0.09 + 0.005 * 4.0), rel=1e-14)
    assert o["mass"] == pytest.approx([M, 0.02], rel=1e-14)
    assert o["volume"][0] == pytest.approx(0.1, rel=1e-14)
    assert o["vmax"] == pytest.approx([0.3, 2.0], rel=1e-14)
    # opposite points of equal mass cancel in the centroid, except the inner
    # pairs (masses 0.01 rho)
    cx = 0.5 + (m[0] - m[1]) * a / M
    cy = 0.5 + (m[2] - m[3]) * a / M
    assert o["centroid"] == pytest.approx([cx, cy], abs=1e-15)
    assert o["r_eq"] == pytest.approx(math.sqrt(0.1 / math.pi), rel=1e-14)
    assert o["p_in"] == pytest.approx((0.1 + 0.2 + 0.3 + 0.4) / 4.0, rel=1e-12)
    assert o["p_out"] == pytest.approx((-0.02 + 0.01) / 2.0, rel=1e-12)
    mxx = (m[0] * (0.5 + a - cx) ** 2 + m[1] * (0.5 - a - cx) ** 2 + (m[2] + m[3]) * (0.5 - cx) ** 2
           + 0.01 * ((0.5 + A - cx) ** 2 + (0.5 - A - cx) ** 2) + 0.02 * (0.5 - cx) ** 2
           + 0.01 * ((0.5 + B - cx) ** 2 + (0.5 - B - cx) ** 2))
    assert o["moment2"][0, 0] == pytest.approx(mxx, rel=1e-12)
    myy = (m[2] * (0.5 + a - cy) ** 2 + m[3] * (0.5 - a - cy) ** 2 + (m[0] + m[1]) * (0.5 - cy) ** 2
           + 0.01 * ((0.5 + A - cy) ** 2 + (0.5 - A - cy) ** 2) + 0.04 * (0.5 - cy) ** 2)
    assert o["moment2"][1, 1] == pytest.approx(myy, rel=1e-12)
    mxy = (m[0] * (a + 0.5 - cx) * (0.5 - cy) + m[1] * (0.5 - a - cx) * (0.5 - cy)
           + m[2] * (0.5 - cx) * (0.5 + a - cy) + m[3] * (0.5 - cx) * (0.5 - a - cy)
           + 0.01 * ((A + 0.5 - cx) + (0.5 - A - cx) + 2 * (0.5 - cx)) * (0.5 - cy)
           + 0.01 * (0.5 - cx) * ((0.5 + A - cy) + (0.5 - A - cy) - 2 * (0.5 - cy))
           + 0.01 * ((B + 0.5 - cx) + (0.5 - B - cx)) * (0.5 - cy))
    assert o["moment2"][0, 1] == pytest.approx(mxy, rel=1e-9, abs=1e-20)
