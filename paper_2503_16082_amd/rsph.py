"""Thin ctypes binding of ``librsph.so`` (C-ABI in ``include/rsph.h``).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module loads the library and raises if it is not built: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsph.so")

FP64 = 0
MIXED = 1

NO_PENALTY = 1
NO_SHIFT = 2
NO_DENSITY_SUMMATION = 4
GBAR_OWN_PHASE_AVERAGE = 8
PENALTY_R3 = 16
NO_SURFACE = 32

KEEP_CLOCK = 1

FIELDS = {
    "pos": 0, "vel": 1, "rho": 2, "p": 3, "drho": 4, "mass": 5, "phase": 6,
    "acc": 7, "acc_p": 8, "acc_s": 9, "acc_v": 10, "gradC": 11, "rate_drho": 12,
    "B": 13, "dr": 14, "sigma": 15, "nnb": 16, "flags": 17,
}
KERNELS = ["bin", "neighbours", "advection", "shift", "colour", "force", "continuity",
           "event_floor"]

HEALTH = {"nonfinite": 1, "density": 2, "neighbours": 4, "coincident": 8, "dt": 32}

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ENUMERIC",
          -6: "EBUSY"}


class RsphError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("precision", C.c_int32),
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
        ("reserved", C.c_uint32),
        ("u_ref", C.c_double),
    ]


class Observables(C.Structure):
    _fields_ = [
        ("t", C.c_double),
        ("n_outer", C.c_int64),
        ("n_sub", C.c_int64),
        ("dt_ad", C.c_double),
        ("dt_ac", C.c_double),
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
        ("health", C.c_uint32),
        ("displaced_steps", C.c_uint32),
    ]


SYMBOLS = [
    "rsph_params_default", "rsph_create_system", "rsph_set_particles", "rsph_set_drho",
    "rsph_step", "rsph_eval_rates", "rsph_read_observables", "rsph_read_particles",
    "rsph_read_binning", "rsph_read_neighbours", "rsph_set_kernel_timing", "rsph_set_launch_mode",
    "rsph_read_kernel_timing", "rsph_destroy_system", "rsph_status_string", "rsph_last_error",
    "rsph_pool_create", "rsph_pool_admit", "rsph_pool_step", "rsph_pool_bytes", "rsph_step_counts",
    "rsph_pool_release", "rsph_pool_destroy", "rsph_eval_rates_noalloc",
]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build()); "
                           "the HIP library is required, there is no fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    L.rsph_params_default.argtypes = [vp]
    L.rsph_params_default.restype = None
    L.rsph_create_system.argtypes = [vp, vp, vp]
    L.rsph_set_particles.argtypes = [vp, i64, vp, vp, vp, vp, vp, u32]
    L.rsph_set_drho.argtypes = [vp, i64, vp]
    L.rsph_step.argtypes = [vp, i64]
    L.rsph_eval_rates.argtypes = [vp]
    L.rsph_read_observables.argtypes = [vp, vp]
    L.rsph_read_particles.argtypes = [vp, i32, i64, vp]
    L.rsph_read_binning.argtypes = [vp, i64, vp, vp]
    L.rsph_read_neighbours.argtypes = [vp, i64, i64, vp, vp]
    L.rsph_set_kernel_timing.argtypes = [vp, i32]
    L.rsph_set_launch_mode.argtypes = [vp, i32]
    L.rsph_read_kernel_timing.argtypes = [vp, vp, vp]
    L.rsph_destroy_system.argtypes = [vp]
    L.rsph_destroy_system.restype = None
    L.rsph_status_string.argtypes = [i32]
    L.rsph_status_string.restype = C.c_char_p
    L.rsph_last_error.argtypes = [vp]
    L.rsph_last_error.restype = C.c_char_p
    L.rsph_pool_create.argtypes = [i32, i32, C.c_size_t, vp, vp]
    L.rsph_pool_admit.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.rsph_pool_step.argtypes = [vp, vp, vp, i32]
    L.rsph_pool_bytes.argtypes = [vp]
    L.rsph_pool_bytes.restype = C.c_size_t
    L.rsph_step_counts.argtypes = [vp, vp, vp, vp]
    L.rsph_pool_release.argtypes = [vp, vp]
    L.rsph_pool_destroy.argtypes = [vp]
    L.rsph_pool_destroy.restype = None
    L.rsph_eval_rates_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    for name in SYMBOLS:
        f = getattr(L, name)
        if f.restype is C.c_int:  # ctypes default
            f.restype = C.c_int32
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(p: dict, precision=None) -> Params:
    q = Params()
    lib().rsph_params_default(C.byref(q))
    q.dim = int(p["dim"])
    q.precision = int(p.get("precision", FP64) if precision is None else precision)
    box = list(p["box"]) + [1.0] * (3 - len(p["box"]))
    q.box = (C.c_double * 3)(*box)
    q.dp = float(p["dp"])
    q.h_over_dp = float(p.get("h_over_dp", 1.3))
    q.rho0 = (C.c_double * 2)(*p["rho0"])
    q.eta = (C.c_double * 2)(*p["eta"])
    q.c0 = float(p["c0"])
    q.gamma = float(p["gamma"])
    q.xi = float(p.get("xi", -1.0))
    q.alpha_shift = float(p.get("alpha_shift", 0.2))
    q.cfl_ad = float(p.get("cfl_ad", 0.1))
    q.cfl_ac = float(p.get("cfl_ac", 0.6))
    g = list(p.get("gravity", [0.0, 0.0, 0.0])) + [0.0] * 3
    q.gravity = (C.c_double * 3)(*g[:3])
    q.flags = int(p.get("flags", 0))
    q.u_ref = float(p.get("u_ref", 0.0))
    return q


def _check(status, handle=None):
    if status != 0:
        msg = lib().rsph_last_error(handle)
        raise RsphError(status, msg.decode() if msg else "")


class System:
    """One simulation (rsph_create_system / rsph_set_particles / rsph_step ...)."""

    def __init__(self, params: dict, precision=None, stream=None, _handle=None, _pool=None):
        self.params = dict(params)
        self.dim = int(params["dim"])
        self._pool = _pool
        if _handle is not None:
            self.h = _handle
            return
        self._prm = make_params(params, precision)
        h = C.c_void_p()
        _check(lib().rsph_create_system(C.byref(self._prm), stream, C.byref(h)))
        self.h = h
        self.n = 0

    def set_particles(self, pos, vel, phase, mass=None, rho=None, keep_clock=False):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        phase = np.ascontiguousarray(phase, dtype=np.int32)
        mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        n = phase.shape[0]
        _check(lib().rsph_set_particles(self.h, n, _p(pos), _p(vel), _p(phase), _p(mass), _p(rho),
                                        KEEP_CLOCK if keep_clock else 0), self.h)
        self.n = n

    def set_drho(self, drho):
        drho = np.ascontiguousarray(drho, dtype=np.float64)
        _check(lib().rsph_set_drho(self.h, drho.shape[0], _p(drho)), self.h)

    def step(self, n_outer=1):
        _check(lib().rsph_step(self.h, int(n_outer)), self.h)

    def eval_rates(self):
        _check(lib().rsph_eval_rates(self.h), self.h)

    def read(self, field):
        d = self.dim
        f = FIELDS[field]
        width = {"pos": d, "vel": d, "acc": d, "acc_p": d, "acc_s": d, "acc_v": d,
                 "gradC": d, "dr": d, "B": d * d}.get(field, 1)
        out = np.zeros(self.n * width)
        _check(lib().rsph_read_particles(self.h, f, self.n, _p(out)), self.h)
        if field == "B":
            return out.reshape(self.n, d, d)
        return out.reshape(self.n, width) if width > 1 else out

    def observables(self):
        o = Observables()
        _check(lib().rsph_read_observables(self.h, C.byref(o)), self.h)
        d = self.dim
        return {
            "t": o.t, "n_outer": o.n_outer, "n_sub": o.n_sub, "dt_ad": o.dt_ad, "dt_ac": o.dt_ac,
            "momentum": np.array(o.momentum[:d]), "kinetic": o.kinetic,
            "mass": np.array(o.mass[:]), "volume": np.array(o.volume[:]),
            "vmax": np.array(o.vmax[:]), "centroid": np.array(o.centroid[:d]),
            "moment2": np.array(o.moment2[:]).reshape(3, 3)[:d, :d], "r_eq": o.r_eq,
            "p_in": o.p_in, "p_out": o.p_out, "n_in": o.n_in, "n_out": o.n_out,
            "health": o.health, "displaced_steps": o.displaced_steps,
        }

    def binning(self):
        key = np.zeros(self.n, np.uint32)
        rank = np.zeros(self.n, np.int64)
        _check(lib().rsph_read_binning(self.h, self.n, _p(key), _p(rank)), self.h)
        return key, rank

    def neighbours(self, cap_per=200):
        start = np.zeros(self.n + 1, np.int64)
        idx = np.zeros(self.n * cap_per, np.int64)
        _check(lib().rsph_read_neighbours(self.h, self.n, idx.shape[0], _p(start), _p(idx)), self.h)
        return start, idx[: start[-1]].copy()

    def step_counts(self):
        """Advection steps, acoustic substeps, and the most substeps one of the
        recent advection steps needed (before the first step an estimate for
        it; after it 0 until a later step is seen), as of the end of the last
        stepping call (host-side; no device access)."""
        out = [C.c_int64() for _ in range(3)]
        _check(lib().rsph_step_counts(self.h, *[C.byref(o) for o in out]), self.h)
        return {"n_outer": out[0].value, "n_sub": out[1].value, "substeps_per_step": out[2].value}

    def set_launch_mode(self, mode):
        """'graph' (captured launch cycles, the default) or 'eager'; applies to
        the whole pool that holds this system."""
        code = {"graph": 0, "eager": 1}[mode]
        _check(lib().rsph_set_launch_mode(self.h, code), self.h)

    def set_timing(self, kernels=None):
        """kernels: iterable of names from KERNELS (None = all, [] = off)."""
        names = KERNELS if kernels is None else list(kernels)
        mask = 0
        for k in names:
            mask |= 1 << KERNELS.index(k)
        _check(lib().rsph_set_kernel_timing(self.h, mask), self.h)

    def timing(self):
        launches = np.zeros(len(KERNELS), np.int64)
        ms = np.zeros(len(KERNELS))
        _check(lib().rsph_read_kernel_timing(self.h, _p(launches), _p(ms)), self.h)
        return {k: (int(launches[i]), float(ms[i])) for i, k in enumerate(KERNELS)}

    def close(self):
        if self.h is not None and self._pool is None:
            lib().rsph_destroy_system(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Packed multi-system pool (rsph_pool_*)."""

    def __init__(self, dim, precision=FP64, budget_bytes=0, stream=None):
        self.dim = dim
        self.precision = precision
        h = C.c_void_p()
        _check(lib().rsph_pool_create(dim, precision, int(budget_bytes), stream, C.byref(h)))
        self.h = h
        self.members = []

    def admit(self, params, pos, vel, phase, mass=None):
        prm = make_params(params, self.precision)
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        phase = np.ascontiguousarray(phase, dtype=np.int32)
        mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        hs = C.c_void_p()
        st = lib().rsph_pool_admit(self.h, C.byref(prm), phase.shape[0], _p(pos), _p(vel),
                                   _p(phase), _p(mass), C.byref(hs))
        if st != 0:
            msg = lib().rsph_last_error(None)
            raise RsphError(st, msg.decode() if msg else "")
        s = System(params, _handle=hs, _pool=self)
        s.n = phase.shape[0]
        self.members.append(s)
        return s

    def step(self, systems, n_outer):
        arr = (C.c_void_p * len(systems))(*[s.h for s in systems])
        n = np.ascontiguousarray(n_outer, dtype=np.int64)
        st = lib().rsph_pool_step(self.h, arr, n.ctypes.data_as(C.c_void_p), len(systems))
        if st != 0:
            msg = lib().rsph_last_error(None)
            raise RsphError(st, msg.decode() if msg else "")

    def release(self, s):
        st = lib().rsph_pool_release(self.h, s.h)
        if st != 0:
            msg = lib().rsph_last_error(None)
            raise RsphError(st, msg.decode() if msg else "")
        self.members.remove(s)
        s.h = None

    def bytes(self):
        return int(lib().rsph_pool_bytes(self.h))

    def close(self):
        if self.h is not None:
            lib().rsph_pool_destroy(self.h)
            for s in self.members:
                s.h = None
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_rates_noalloc(params, n, pos, vel, phase, acc, drho, mass=None, rho=None, precision=None, stream=None):
    """rsph_eval_rates_noalloc on caller-owned device buffers, given by their
    device addresses (integers, e.g. torch's data_ptr()); mass and rho may be
    None.  Raises RsphError on a non-zero status."""
    prm = make_params(params, precision)
    st = lib().rsph_eval_rates_noalloc(C.byref(prm), int(n), C.c_void_p(pos), C.c_void_p(vel),
                                       C.c_void_p(phase), None if mass is None else C.c_void_p(mass),
                                       None if rho is None else C.c_void_p(rho), C.c_void_p(acc),
                                       C.c_void_p(drho), None if stream is None else C.c_void_p(stream))
    if st != 0:
        msg = lib().rsph_last_error(None)
        raise RsphError(st, msg.decode() if msg else "")
