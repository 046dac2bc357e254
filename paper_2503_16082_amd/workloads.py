"""Seeded synthetic droplet workloads (inputs only).

This module builds initial particle sets and parameter dictionaries for the
workloads the method is exercised on: a lattice of spacing dp in a periodic box,
seeded uniform jitter of 0.05 dp, a phase assigned from the unjittered lattice
point, and zero or prescribed velocity.  It holds none of the method's
arithmetic: it draws random numbers and lays out lattices, nothing more, so it
can feed both the HIP library and the CPU oracle with identical arrays.

Phase 0 is fluid k (the droplet or pool), phase 1 is fluid l, phase 2 a wall
particle (fixed; its velocity is the wall's).  The sound speed
follows the paper's rule c0 = 10 U (section 2), with U the larger of the initial
speed and the capillary velocity sqrt((d-1) gamma / (rho_k R)).
"""
from __future__ import annotations

import math

import numpy as np

H_OVER_DP = 1.3


def lattice(dim, counts, dp):
    """Cell-centred lattice ((i + 1/2) dp, ...), x fastest."""
    axes = [(np.arange(c) + 0.5) * dp for c in counts]
    grids = np.meshgrid(*axes[::-1], indexing="ij")
    pts = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    return pts.astype(np.float64)


def jitter(rng, pts, dp, amp=0.05):
    return pts + rng.uniform(-amp * dp, amp * dp, size=pts.shape)


def base_params(dim, box, dp, rho0, eta, gamma, c0, **kw):
    p = {
        "dim": dim,
        "box": [float(b) for b in box],
        "dp": float(dp),
        "h_over_dp": H_OVER_DP,
        "rho0": [float(rho0[0]), float(rho0[1])],
        "eta": [float(eta[0]), float(eta[1])],
        "gamma": float(gamma),
        "c0": float(c0),
        "xi": -1.0,
        "alpha_shift": 0.2,
        "cfl_ad": 0.1,
        "cfl_ac": 0.6,
        "gravity": [0.0, 0.0, 0.0],
    }
    p.update(kw)
    return p


def capillary_c0(dim, gamma, rho_k, R, umax=0.0):
    return 10.0 * max(umax, math.sqrt((dim - 1) * gamma / (rho_k * R)))


def static_droplet_2d(n_side=50, R=0.2, seed=0, rho=(1000.0, 1.0), eta=(0.1, 1e-3),
                      gamma=1.0, amp=0.05):
    """Disc of radius R centred in the periodic unit square (2,500 particles at
    n_side = 50)."""
    dp = 1.0 / n_side
    pts0 = lattice(2, (n_side, n_side), dp)
    phase = np.where(np.linalg.norm(pts0 - 0.5, axis=1) < R, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    p = base_params(2, (1.0, 1.0), dp, rho, eta, gamma, capillary_c0(2, gamma, rho[0], R))
    return {"name": "static_droplet_2d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": R}


def square_droplet_2d(n_side=200, side=0.4, seed=0, rho=(1000.0, 1.0), eta=(0.1, 1e-3),
                      gamma=1.0, amp=0.05):
    """Square of the given side centred in the periodic unit square (40,000
    particles at n_side = 200)."""
    dp = 1.0 / n_side
    pts0 = lattice(2, (n_side, n_side), dp)
    inside = np.max(np.abs(pts0 - 0.5), axis=1) < 0.5 * side
    phase = np.where(inside, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    R = side / math.sqrt(math.pi)
    p = base_params(2, (1.0, 1.0), dp, rho, eta, gamma, capillary_c0(2, gamma, rho[0], R))
    return {"name": "square_droplet_2d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": R}


def static_droplet_3d(n_side=64, R=0.25, seed=0, rho=(1000.0, 1.0), eta=(0.1, 1e-3),
                      gamma=1.0, amp=0.05):
    """Sphere of radius R centred in the periodic unit cube (262,144 particles at
    n_side = 64)."""
    dp = 1.0 / n_side
    pts0 = lattice(3, (n_side, n_side, n_side), dp)
    phase = np.where(np.linalg.norm(pts0 - 0.5, axis=1) < R, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    p = base_params(3, (1.0, 1.0, 1.0), dp, rho, eta, gamma,
                    capillary_c0(3, gamma, rho[0], R))
    return {"name": "static_droplet_3d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": R, "n_side": n_side}


def subset_indices_3d(n_side, lo, hi):
    """Indices of the lattice block lo <= (ix, iy, iz) < hi (x fastest)."""
    ix = np.arange(lo[0], hi[0])
    iy = np.arange(lo[1], hi[1])
    iz = np.arange(lo[2], hi[2])
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    return (X + n_side * (Y + n_side * Z)).ravel().astype(np.int64)


def oscillating_ellipse_2d(n_particles, aspect, ratio, gamma, seed, R=0.2, rho_k=1000.0,
                           eta_k=0.1, amp=0.05):
    """One served job: an ellipse of semi-axes R sqrt(AR), R / sqrt(AR) in the
    periodic unit square, round(sqrt(N)) particles per side."""
    n_side = max(3, int(round(math.sqrt(n_particles))))
    dp = 1.0 / n_side
    pts0 = lattice(2, (n_side, n_side), dp)
    a = R * math.sqrt(aspect)
    b = R / math.sqrt(aspect)
    x = (pts0[:, 0] - 0.5) / a
    y = (pts0[:, 1] - 0.5) / b
    phase = np.where(x * x + y * y < 1.0, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    rho = (rho_k, rho_k / ratio)
    eta = (eta_k, eta_k / min(ratio, 100.0))
    p = base_params(2, (1.0, 1.0), dp, rho, eta, gamma, capillary_c0(2, gamma, rho_k, R))
    return {"name": "oscillating_ellipse_2d", "params": p, "pos": pos, "vel": vel,
            "phase": phase, "R": R}


def oscillating_drop_2d(n_side=60, ratio=1000.0, V0=1.0, gamma=1.0, seed=0, R=0.2, r0=0.05, rho_k=1.0,
                        eta_k=0.05, amp=0.05):
    """Oscillating drop of section 5.1: a disc of radius R centred in the
    periodic unit square, started with the divergence-free velocity field of
    Eq. 34 (centred on the drop, scale r0) on every particle.  Phase k has
    rho_k, eta_k; phase l has rho_k / ratio and eta_k / min(ratio, 100)
    (ratio 1000: rho 1e-3, eta 5e-4).  n_side = 60 gives R / dp = 12."""
    dp = 1.0 / n_side
    pts0 = lattice(2, (n_side, n_side), dp)
    d0 = pts0 - 0.5
    phase = np.where((d0 * d0).sum(axis=1) < R * R, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    x = pos[:, 0] - 0.5
    y = pos[:, 1] - 0.5
    r = np.sqrt(x * x + y * y)
    decay = np.exp(-r / r0)
    rs = np.maximum(r, 1e-300)
    vel = np.stack([V0 * (x / r0) * (1.0 - y * y / (r0 * rs)) * decay,
                    -V0 * (y / r0) * (1.0 - x * x / (r0 * rs)) * decay], axis=1)
    umax = float(np.sqrt((vel * vel).sum(axis=1)).max())
    rho = (rho_k, rho_k / ratio)
    eta = (eta_k, eta_k / min(ratio, 100.0))
    p = base_params(2, (1.0, 1.0), dp, rho, eta, gamma, capillary_c0(2, gamma, rho_k, R, umax))
    return {"name": "oscillating_drop_2d", "params": p, "pos": pos, "vel": vel, "phase": phase, "R": R}


def served_mix(n_jobs=256, seed=0, n_min=2000, n_max=200000):
    """Job descriptions of the served mix: log-uniform particle counts,
    aspect ratio U(1.1, 1.5), density ratio from {10, 100, 1000}, gamma U(0.5, 2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for k in range(n_jobs):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        jobs.append({
            "job": k,
            "n": n,
            "aspect": float(rng.uniform(1.1, 1.5)),
            "ratio": float(rng.choice([10.0, 100.0, 1000.0])),
            "gamma": float(rng.uniform(0.5, 2.0)),
            "seed": k,
        })
    return jobs


def droplet_impact_3d(n_per_unit=32, seed=0, U0=50.0, amp=0.05, box=(8.0, 8.0, 4.0),
                      pool_depth=2.0, D=1.0):
    """Droplet of diameter D with velocity (0, 0, -U0) just above a pool of depth
    pool_depth in a fully periodic air-filled box (8,388,608 particles at 32
    per unit length)."""
    dp = 1.0 / n_per_unit
    counts = tuple(int(round(b / dp)) for b in box)
    pts0 = lattice(3, counts, dp)
    centre = np.array([box[0] / 2, box[1] / 2, pool_depth + D / 2 + 2 * dp])
    in_drop = np.linalg.norm(pts0 - centre, axis=1) < D / 2
    in_pool = pts0[:, 2] < pool_depth
    phase = np.where(in_drop | in_pool, 0, 1).astype(np.int32)
    del pts0
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = lattice(3, counts, dp)
    pos += rng.uniform(-amp * dp, amp * dp, size=pos.shape)
    vel = np.zeros_like(pos)
    vel[in_drop, 2] = -U0
    p = base_params(3, box, dp, (1.0, 1e-3), (5e-3, 5e-5), 0.1, 10.0 * U0)
    return {"name": "droplet_impact_3d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": D / 2, "centre": centre, "pool_depth": pool_depth}


def acoustic_wave_2d(n_side=24, amp_v=1e-3, seed=0):
    """Single-phase periodic box with a sinusoidal velocity perturbation, used
    to check that the Riemann dissipation damps acoustic energy."""
    dp = 1.0 / n_side
    pos = lattice(2, (n_side, n_side), dp)
    vel = np.zeros_like(pos)
    vel[:, 0] = amp_v * np.sin(2 * math.pi * pos[:, 0])
    phase = np.zeros(pos.shape[0], np.int32)
    p = base_params(2, (1.0, 1.0), dp, (1.0, 1.0), (0.0, 0.0), 0.0, 0.1)
    return {"name": "acoustic_wave_2d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": 0.0}


WALL = 2
WALL_LAYERS = 3  # 3 dp of wall behind a wall face covers the 2.6 dp kernel support


def with_walls(pos, vel, phase, box, dp, axis, v_lo=None, v_hi=None, layers=WALL_LAYERS):
    """Closes a periodic box along `axis` with two walls: every particle moves
    up by layers * dp, and lattice layers of wall particles fill [0, layers dp)
    and [L + layers dp, L + 2 layers dp), where L is the box's old length along
    the axis; the box grows to L + 2 layers dp.  The two walls' outer layers
    meet across the periodic boundary, so no fluid particle sees through a
    wall.  v_lo, v_hi: the walls' velocities (default at rest).  Returns
    (pos, vel, phase, box)."""
    dim = pos.shape[1]
    box = [float(b) for b in box]
    L = box[axis]
    counts = [int(round(b / dp)) for b in box]
    counts[axis] = layers
    slab = lattice(dim, counts, dp)
    lo = slab.copy()
    hi = slab.copy()
    hi[:, axis] += L + layers * dp
    pos = pos.copy()
    pos[:, axis] += layers * dp
    wv = np.zeros((2 * len(slab), dim))
    if v_lo is not None:
        wv[:len(slab)] = np.asarray(v_lo, dtype=np.float64)
    if v_hi is not None:
        wv[len(slab):] = np.asarray(v_hi, dtype=np.float64)
    box[axis] = L + 2 * layers * dp
    return (np.vstack([pos, lo, hi]), np.vstack([vel, wv]),
            np.concatenate([phase, np.full(2 * len(slab), WALL, np.int32)]).astype(np.int32), box)


def droplet_impact_wall_3d(n_per_unit=32, seed=0, U0=50.0, amp=0.05, box=(8.0, 8.0, 1.5), D=1.0):
    """The high-velocity impact of section 5.4: a drop of diameter D (fluid k,
    rho 1, eta 0.005, gamma 0.1, velocity (0, 0, -U0)) in air (rho 1e-3, eta
    5e-5) in an 8 x 8 x 1.5 box whose floor the drop's bottom touches; walls at
    the floor and the ceiling, periodic sides.  U0 = 50 gives Re = 1e4 and
    We = 2.5e4 (Eq. 38).  At 32 particles per unit length: 3,145,728 fluid
    particles and 393,216 wall particles."""
    dp = 1.0 / n_per_unit
    counts = tuple(int(round(b / dp)) for b in box)
    pts0 = lattice(3, counts, dp)
    centre = np.array([box[0] / 2, box[1] / 2, D / 2])
    in_drop = np.linalg.norm(pts0 - centre, axis=1) < D / 2
    phase = np.where(in_drop, 0, 1).astype(np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    vel[in_drop, 2] = -U0
    pos, vel, phase, box3 = with_walls(pos, vel, phase, box, dp, axis=2)
    p = base_params(3, box3, dp, (1.0, 1e-3), (5e-3, 5e-5), 0.1, 10.0 * U0)
    return {"name": "droplet_impact_wall_3d", "params": p, "pos": pos, "vel": vel, "phase": phase,
            "R": D / 2, "centre": centre + np.array([0.0, 0.0, WALL_LAYERS * dp])}


def channel_2d(n_side=20, seed=0, rho=(1.0, 1.0), eta=(0.05, 0.05), v_wall=0.0, gamma=0.0, c0=1.0, amp=0.05):
    """Fluid k filling a 1 x 1 periodic square closed by walls along y (the
    bottom at rest, the top moving with (v_wall, 0)): the setting of the wall
    checks and of the Couette shear of section 5.2."""
    dp = 1.0 / n_side
    pts0 = lattice(2, (n_side, n_side), dp)
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = jitter(rng, pts0, dp, amp)
    vel = np.zeros_like(pos)
    phase = np.zeros(len(pos), np.int32)
    pos, vel, phase, box = with_walls(pos, vel, phase, (1.0, 1.0), dp, axis=1, v_hi=(v_wall, 0.0))
    p = base_params(2, box, dp, rho, eta, gamma, c0)
    return {"name": "channel_2d", "params": p, "pos": pos, "vel": vel, "phase": phase, "R": 0.0}
