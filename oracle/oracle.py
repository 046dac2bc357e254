"""Python binding of the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path.  The library is
compiled from ``rsph_oracle.c`` by the repository's build step; this module only
marshals numpy arrays into it.

Every function mirrors one C entry point; the method's arithmetic lives in C.
Particle arrays are row-major ``(n, dim)`` float64; phases are int32 in {0, 1, 2}
(0 = fluid k, the droplet; 1 = fluid l; 2 = a wall particle, which never moves).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RSPH_ORACLE_LIB points the binding at another build of the same source
LIB_PATH = os.environ.get("RSPH_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

NO_PENALTY = 1
NO_SHIFT = 2
NO_DENSITY_SUMMATION = 4
GBAR_OWN_PHASE_AVERAGE = 8
PENALTY_R3 = 16
NO_SURFACE = 32
WALL = 2


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("reserved", C.c_int32),
        ("box", C.c_double * 3),
        ("dp", C.c_double),
        ("h_over_dp", C.c_double),
        ("rho0", C.c_double * 2),
        ("eta", C.c_double * 2),
        ("c0", C.c_double),
        ("gamma", C.c_double),
        ("xi", C.c_double),
        ("alpha_shift", C.c_double),
        ("cfl_ad", C.c_double),
        ("cfl_ac", C.c_double),
        ("gravity", C.c_double * 3),
        ("flags", C.c_uint32),
        ("reserved2", C.c_uint32),
    ]


class OrcClock(C.Structure):
    _fields_ = [
        ("t", C.c_double),
        ("dt_ad", C.c_double),
        ("dt_ac", C.c_double),
        ("n_outer", C.c_double),
        ("n_sub", C.c_double),
        ("vmax", C.c_double * 2),
    ]


class OrcRates(C.Structure):
    _fields_ = [
        ("gradC", C.c_void_p),
        ("acc", C.c_void_p),
        ("acc_p", C.c_void_p),
        ("acc_s", C.c_void_p),
        ("acc_v", C.c_void_p),
        ("drho", C.c_void_p),
        ("B", C.c_void_p),
        ("dr", C.c_void_p),
        ("sigma", C.c_void_p),
        ("nnb", C.c_void_p),
    ]


class OrcObs(C.Structure):
    _fields_ = [
        ("momentum", C.c_double * 3),
        ("kinetic", C.c_double),
        ("mass", C.c_double * 2),
        ("volume", C.c_double * 2),
        ("vmax", C.c_double * 2),
        ("centroid", C.c_double * 3),
        ("moment2", C.c_double * 9),
        ("r_eq", C.c_double),
        ("p_in", C.c_double),
        ("p_out", C.c_double),
        ("n_in", C.c_double),
        ("n_out", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.orc_W.restype = d
        L.orc_W.argtypes = [i32, d, d]
        L.orc_dW.restype = d
        L.orc_dW.argtypes = [i32, d, d]
        L.orc_sigma0.restype = d
        L.orc_sigma0.argtypes = [i32, d, d]
        L.orc_xi_auto.restype = d
        L.orc_xi_auto.argtypes = [d, d]
        L.orc_grid.restype = i32
        L.orc_grid.argtypes = [vp, vp]
        L.orc_wrap_positions.restype = None
        L.orc_wrap_positions.argtypes = [vp, i64, vp]
        L.orc_cell_keys.restype = None
        L.orc_cell_keys.argtypes = [vp, i64, vp, vp]
        L.orc_bin.restype = None
        L.orc_bin.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_neighbours_brute.restype = i64
        L.orc_neighbours_brute.argtypes = [vp, i64, vp, vp, vp, i64]
        L.orc_neighbours_cells.restype = i64
        L.orc_neighbours_cells.argtypes = [vp, i64, vp, vp, vp, i64]
        L.orc_eval_rates.restype = i32
        L.orc_eval_rates.argtypes = [vp, i64, vp, vp, vp, vp, vp, i64, vp, vp]
        L.orc_step.restype = i32
        L.orc_step.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, i64]
        L.orc_observables.restype = None
        L.orc_observables.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.orc_dt_advection.restype = d
        L.orc_dt_advection.argtypes = [vp, vp]
        L.orc_dt_acoustic.restype = d
        L.orc_dt_acoustic.argtypes = [vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(p: dict) -> OrcParams:
    """Builds the C parameter record from a parameter dictionary."""
    o = OrcParams()
    o.dim = int(p["dim"])
    box = list(p["box"]) + [0.0] * (3 - len(p["box"]))
    o.box = (C.c_double * 3)(*box)
    o.dp = float(p["dp"])
    o.h_over_dp = float(p.get("h_over_dp", 1.3))
    o.rho0 = (C.c_double * 2)(*p["rho0"])
    o.eta = (C.c_double * 2)(*p["eta"])
    o.c0 = float(p["c0"])
    o.gamma = float(p["gamma"])
    o.xi = float(p.get("xi", -1.0))
    o.alpha_shift = float(p.get("alpha_shift", 0.2))
    o.cfl_ad = float(p.get("cfl_ad", 0.1))
    o.cfl_ac = float(p.get("cfl_ac", 0.6))
    g = list(p.get("gravity", [0.0, 0.0, 0.0])) + [0.0] * 3
    o.gravity = (C.c_double * 3)(*g[:3])
    o.flags = int(p.get("oracle_flags", 0))
    return o


def W(dim, h, r):
    return lib().orc_W(dim, h, r)


def dW(dim, h, r):
    return lib().orc_dW(dim, h, r)


def sigma0(dim, h, dp):
    return lib().orc_sigma0(dim, h, dp)


def xi_auto(rho_a, rho_b):
    return lib().orc_xi_auto(rho_a, rho_b)


def grid(p):
    P = make_params(p)
    nc = np.zeros(3, np.int32)
    ok = lib().orc_grid(C.byref(P), _ptr(nc))
    return bool(ok), nc


def wrap(p, pos):
    P = make_params(p)
    out = np.ascontiguousarray(pos, dtype=np.float64).copy()
    lib().orc_wrap_positions(C.byref(P), out.shape[0], _ptr(out))
    return out


def cell_keys(p, pos):
    P = make_params(p)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    key = np.zeros(pos.shape[0], np.uint32)
    lib().orc_cell_keys(C.byref(P), pos.shape[0], _ptr(pos), _ptr(key))
    return key


def bin_particles(p, key, pos):
    """Counting sort by cell key, each cell ordered by (x, index): returns
    (perm, cell_start)."""
    P = make_params(p)
    ok, nc = grid(p)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    assert pos.shape == (key.shape[0], p["dim"])
    perm = np.zeros(key.shape[0], np.int64)
    cs = np.zeros(int(np.prod(nc)) + 1, np.int64)
    lib().orc_bin(C.byref(P), key.shape[0], _ptr(key), _ptr(pos), _ptr(perm), _ptr(cs))
    return perm, cs


def _neighbours(fn, p, pos, cap_per=200):
    P = make_params(p)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    start = np.zeros(n + 1, np.int64)
    cap = max(1, n * cap_per)
    idx = np.zeros(cap, np.int64)
    tot = fn(C.byref(P), n, _ptr(pos), _ptr(start), _ptr(idx), cap)
    if tot < 0:
        raise RuntimeError("neighbour capacity exceeded")
    return start, idx[:tot].copy()


def neighbours_brute(p, pos, cap_per=200):
    """O(N^2) neighbour lists (CSR, ascending j). Positions must be wrapped."""
    return _neighbours(lib().orc_neighbours_brute, p, pos, cap_per)


def neighbours_cells(p, pos, cap_per=200):
    """Cell-list neighbour lists (CSR, ascending j). Positions must be wrapped."""
    return _neighbours(lib().orc_neighbours_cells, p, pos, cap_per)


def eval_rates(p, pos, vel, rho, mass, phase, targets=None):
    """One evaluation of every rate at the state given; positions must be
    wrapped. Returns a dict of arrays over the targets (all particles when
    targets is None)."""
    P = make_params(p)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    phase = np.ascontiguousarray(phase, dtype=np.int32)
    n = pos.shape[0]
    if targets is not None:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt = targets.shape[0]
    else:
        nt = n
    out = {
        "gradC": np.zeros((nt, 3)),
        "acc": np.zeros((nt, 3)),
        "acc_p": np.zeros((nt, 3)),
        "acc_s": np.zeros((nt, 3)),
        "acc_v": np.zeros((nt, 3)),
        "drho": np.zeros(nt),
        "B": np.zeros((nt, 9)),
        "dr": np.zeros((nt, 3)),
        "sigma": np.zeros(nt),
        "nnb": np.zeros(nt, np.int64),
    }
    R = OrcRates(*[_ptr(out[k]) for k in
                   ["gradC", "acc", "acc_p", "acc_s", "acc_v", "drho", "B", "dr",
                    "sigma", "nnb"]])
    rc = lib().orc_eval_rates(C.byref(P), n, _ptr(pos), _ptr(vel), _ptr(rho), _ptr(mass),
                              _ptr(phase), nt, _ptr(targets), C.byref(R))
    if rc != 0:
        raise RuntimeError("oracle eval_rates failed (neighbour overflow)")
    d = int(p["dim"])
    for k in ["gradC", "acc", "acc_p", "acc_s", "acc_v", "dr"]:
        out[k] = out[k][:, :d]
    out["B"] = out["B"][:, : d * d].reshape(nt, d, d)
    return out


class State:
    """Host-side state advanced by the oracle's time integrator."""

    def __init__(self, p, pos, vel, phase, mass=None, rho=None):
        self.p = dict(p)
        d = int(p["dim"])
        self.pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, d).copy()
        n = self.pos.shape[0]
        self.vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(n, d).copy()
        self.phase = np.ascontiguousarray(phase, dtype=np.int32).copy()
        # fluid ids 0 and 1 are the fluids k and l, 2 marks a wall particle
        # (reference density 1, so that its volume is the lattice volume)
        rho0 = np.asarray(list(p["rho0"]) + [1.0], dtype=np.float64)
        if mass is None:
            h = p["dp"] * p.get("h_over_dp", 1.3)
            mass = rho0[self.phase] / sigma0(d, h, p["dp"])
        self.mass = np.ascontiguousarray(mass, dtype=np.float64).copy()
        self.rho = (rho0[self.phase].copy() if rho is None
                    else np.ascontiguousarray(rho, dtype=np.float64).copy())
        self.drho = np.zeros(n)
        self.clock = OrcClock()

    def step(self, n_outer):
        P = make_params(self.p)
        rc = lib().orc_step(C.byref(P), self.pos.shape[0], _ptr(self.pos), _ptr(self.vel),
                            _ptr(self.rho), _ptr(self.drho), _ptr(self.mass),
                            _ptr(self.phase), C.byref(self.clock), int(n_outer))
        if rc != 0:
            raise RuntimeError(f"oracle step failed ({rc})")

    def observables(self):
        P = make_params(self.p)
        o = OrcObs()
        lib().orc_observables(C.byref(P), self.pos.shape[0], _ptr(self.pos), _ptr(self.vel),
                              _ptr(self.rho), _ptr(self.mass), _ptr(self.phase), C.byref(o))
        d = int(self.p["dim"])
        return {
            "t": self.clock.t,
            "n_outer": int(self.clock.n_outer),
            "n_sub": int(self.clock.n_sub),
            "dt_ad": self.clock.dt_ad,
            "dt_ac": self.clock.dt_ac,
            "momentum": np.array(o.momentum[:d]),
            "kinetic": o.kinetic,
            "mass": np.array(o.mass[:]),
            "volume": np.array(o.volume[:]),
            "vmax": np.array(o.vmax[:]),
            "centroid": np.array(o.centroid[:d]),
            "moment2": np.array(o.moment2[:]).reshape(3, 3)[:d, :d],
            "r_eq": o.r_eq,
            "p_in": o.p_in,
            "p_out": o.p_out,
        }


def dt_advection(p, vmax):
    P = make_params(p)
    v = np.ascontiguousarray(vmax, dtype=np.float64)
    return lib().orc_dt_advection(C.byref(P), _ptr(v))


def dt_acoustic(p, vmax):
    P = make_params(p)
    v = np.ascontiguousarray(vmax, dtype=np.float64)
    return lib().orc_dt_acoustic(C.byref(P), _ptr(v))
