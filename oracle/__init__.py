"""CPU oracle for the direct N-body hot path (ctypes over liboracle.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product library never does.  The
arithmetic lives in nbody_oracle.c (plain FP64 C, compensated sums); this
module only marshals numpy arrays.  See that file for the definitions and
the passages of the paper they follow.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB points the package at another build of the same source: the
# mutation test loads copies with planted mistakes this way
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

TICK_BITS = 20
OK, EINVAL, ENONFINITE, EDOMAIN = 0, -1, -6, -7


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


FIELD_KEYS = ("bulge_m", "bulge_b", "disk_m", "disk_a", "disk_b", "halo_m", "halo_a",
              "halo_gamma", "halo_rc")


class Field(C.Structure):
    """External (Galactic) field parameters; see oracle_field_eval."""
    _fields_ = [(k, C.c_double) for k in FIELD_KEYS]


def make_field(field):
    """A Field from a dict of FIELD_KEYS (missing components are off), or None."""
    if field is None:
        return None
    unknown = set(field) - set(FIELD_KEYS)
    if unknown:
        raise ValueError(f"unknown field keys {sorted(unknown)}")
    return Field(*[float(field.get(k, 0.0)) for k in FIELD_KEYS])


def _fp(f):
    return C.byref(f) if f is not None else None


class Params(C.Structure):
    _fields_ = [("eps", C.c_double), ("eta", C.c_double),
                ("eta_start", C.c_double), ("dt_shared", C.c_double),
                ("level_min", C.c_int32), ("level_max", C.c_int32),
                ("field", C.POINTER(Field))]


class Stats(C.Structure):
    _fields_ = [("n_block_steps", C.c_int64), ("n_interactions", C.c_int64),
                ("n_floor", C.c_int64), ("t_tick", C.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.oracle_forces.argtypes = [C.c_int64, P, C.c_int64, P, P, P, C.c_double, P, P, P]
        L.oracle_energy.argtypes = [C.c_int64, P, P, P, C.c_double, P, P]
        L.oracle_field_eval.argtypes = [P, P, P, P, P, P]
        L.oracle_field_eval.restype = None
        L.oracle_field_all.argtypes = [P, C.c_int64, P, P, P, P, P]
        L.oracle_field_all.restype = None
        L.oracle_predict_one.argtypes = [P, P, P, P, C.c_double, P, P]
        L.oracle_predict_one.restype = None
        L.oracle_predict.argtypes = [C.c_int64, P, P, P, P, P, P, P]
        L.oracle_predict.restype = None
        L.oracle_correct_one.argtypes = [P, P, P, P, P, P, C.c_double, P, P, P, P]
        L.oracle_correct_one.restype = None
        L.oracle_aarseth_dt.argtypes = [P, P, P, P, C.c_double]
        L.oracle_aarseth_dt.restype = C.c_double
        L.oracle_next_level.argtypes = [C.c_int, C.c_double, C.c_int64, C.c_int, C.c_int, P]
        L.oracle_initial_level.argtypes = [P, P, C.c_double, C.c_int, C.c_int, P]
        L.oracle_init.argtypes = [C.c_int64, P, P, P, P, P, P, P, P, P]
        L.oracle_run.argtypes = [C.c_int64, P, P, P, P, P, P, P, P, C.c_int64, C.c_int64, P]
        L.oracle_threads.argtypes = []
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_symplectic_weights.argtypes = [C.c_int, P]
        L.oracle_symplectic.argtypes = [C.c_int64, P, P, P, C.c_double, P, C.c_double,
                                        C.c_int64, C.c_int]
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def forces(x, v, m, eps, idx=None, want_pot=False):
    """Acceleration and jerk (and potential) on particles idx of the set
    (x, v, m).  Returns acc (n_i, 3), jerk (n_i, 3)[, pot (n_i,)]."""
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (n, 3))
    v = _f64(v, (n, 3))
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, np.int64)
    ni = idx.shape[0]
    acc = np.empty((ni, 3))
    jerk = np.empty((ni, 3))
    pot = np.empty(ni) if want_pot else None
    rc = lib().oracle_forces(ni, _p(idx), n, _p(x), _p(v), _p(m), float(eps),
                             _p(acc), _p(jerk), _p(pot) if want_pot else None)
    if rc:
        raise OracleError(rc, "forces")
    return (acc, jerk, pot) if want_pot else (acc, jerk)


LEAPFROG, SYMPLECTIC6 = 0, 1


def symplectic_weights(scheme):
    """Stage weights of the leapfrog (0) or the sixth-order scheme (1)."""
    w = np.empty(7)
    k = lib().oracle_symplectic_weights(int(scheme), _p(w))
    if k == 0:
        raise OracleError(EINVAL, "symplectic_weights")
    return w[:k].copy()


def symplectic(x, v, m, eps, h, n_steps, scheme, field=None):
    """n_steps steps of size h of a symplectic driver (with the external
    field given as a dict of FIELD_KEYS, or none); returns new (x, v)."""
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    f = make_field(field)
    rc = lib().oracle_symplectic(n, _p(m), _p(x), _p(v), float(eps), _fp(f), float(h),
                                 int(n_steps), int(scheme))
    if rc:
        raise OracleError(rc, "symplectic")
    return x, v


def energy(x, v, m, eps, field=None):
    """{K, W, E, L(3), P(3)} of one system; E includes the external field's
    potential energy when a field is given."""
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (n, 3))
    v = _f64(v, (n, 3))
    out = np.empty(9)
    f = make_field(field)
    rc = lib().oracle_energy(n, _p(x), _p(v), _p(m), float(eps), _fp(f), _p(out))
    if rc:
        raise OracleError(rc, "energy")
    return {"K": out[0], "W": out[1], "E": out[2], "L": out[3:6].copy(),
            "P": out[6:9].copy()}


def field_eval(field, x, v):
    """External field on points x with velocities v ((n, 3) or (3,)):
    returns (acc, jerk, pot) of matching shapes."""
    f = make_field(field)
    x = np.asarray(x, np.float64)
    single = x.ndim == 1
    x = _f64(x.reshape(-1, 3))
    n = x.shape[0]
    v = _f64(np.asarray(v, np.float64).reshape(-1, 3), (n, 3))
    acc, jerk, pot = np.empty((n, 3)), np.empty((n, 3)), np.empty(n)
    lib().oracle_field_all(C.byref(f), n, _p(x), _p(v), _p(acc), _p(jerk), _p(pot))
    if single:
        return acc[0], jerk[0], pot[0]
    return acc, jerk, pot


def predict_one(x, v, a, j, dt):
    xs = [_f64(q, (3,)) for q in (x, v, a, j)]
    xp, vp = np.empty(3), np.empty(3)
    lib().oracle_predict_one(*[_p(q) for q in xs], float(dt), _p(xp), _p(vp))
    return xp, vp


def predict(x, v, a, j, dt):
    """Predict every particle over its own interval dt (scalar or (n,))."""
    x = _f64(x)
    n = x.shape[0]
    v, a, j = (_f64(q, (n, 3)) for q in (v, a, j))
    dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (n,)))
    xp, vp = np.empty((n, 3)), np.empty((n, 3))
    lib().oracle_predict(n, _p(x), _p(v), _p(a), _p(j), _p(dt), _p(xp), _p(vp))
    return xp, vp


def correct_one(xp, vp, a0, j0, a1, j1, h):
    ins = [_f64(q, (3,)) for q in (xp, vp, a0, j0, a1, j1)]
    outs = [np.empty(3) for _ in range(4)]
    lib().oracle_correct_one(*[_p(q) for q in ins], float(h), *[_p(q) for q in outs])
    return tuple(outs)   # x1, v1, a2_end, a3


def aarseth_dt(a, j, a2, a3, eta):
    ins = [_f64(q, (3,)) for q in (a, j, a2, a3)]
    return lib().oracle_aarseth_dt(*[_p(q) for q in ins], float(eta))


def next_level(level, dt_c, t_tick, level_min, level_max):
    nf = C.c_int64(0)
    lv = lib().oracle_next_level(int(level), float(dt_c), int(t_tick), int(level_min),
                                 int(level_max), C.byref(nf))
    return lv, nf.value


def initial_level(a, j, eta_s, level_min, level_max):
    nf = C.c_int64(0)
    lv = lib().oracle_initial_level(_p(_f64(a, (3,))), _p(_f64(j, (3,))), float(eta_s),
                                    int(level_min), int(level_max), C.byref(nf))
    return lv, nf.value


class System:
    """Hermite-4 block-step state of one isolated system (oracle side)."""

    def __init__(self, m, x, v, eps, eta=0.01, eta_start=0.01, dt_shared=0.0,
                 level_min=3, level_max=20, field=None):
        self.m = _f64(m).copy()
        n = self.m.shape[0]
        self.x = _f64(x, (n, 3)).copy()
        self.v = _f64(v, (n, 3)).copy()
        self.a = np.empty((n, 3))
        self.j = np.empty((n, 3))
        self.tick = np.zeros(n, np.int64)
        self.level = np.zeros(n, np.int8)
        self.field_dict = dict(field) if field is not None else None
        self._field = make_field(field)          # kept alive for the params pointer
        self.params = Params(float(eps), float(eta), float(eta_start), float(dt_shared),
                             int(level_min), int(level_max),
                             C.pointer(self._field) if self._field is not None else None)
        self.stats = Stats()
        rc = lib().oracle_init(n, _p(self.m), _p(self.x), _p(self.v), C.byref(self.params),
                               _p(self.a), _p(self.j), _p(self.tick), _p(self.level),
                               C.byref(self.stats))
        if rc:
            raise OracleError(rc, "init")

    @property
    def n(self):
        return self.m.shape[0]

    @property
    def t(self):
        return self.stats.t_tick / float(1 << TICK_BITS)

    def run(self, t_end, max_steps=0):
        t_tick = int(round(t_end * (1 << TICK_BITS)))
        if t_tick != t_end * (1 << TICK_BITS):
            raise ValueError("t_end must be a multiple of 2^-20")
        rc = lib().oracle_run(self.n, _p(self.m), _p(self.x), _p(self.v), _p(self.a),
                              _p(self.j), _p(self.tick), _p(self.level),
                              C.byref(self.params), t_tick, int(max_steps),
                              C.byref(self.stats))
        if rc:
            raise OracleError(rc, "run")
        return self

    def energy(self):
        return energy(self.x, self.v, self.m, self.params.eps, self.field_dict)


def threads() -> int:
    return lib().oracle_threads()


def set_threads(n: int):
    """Threads for later oracle calls (results do not depend on it)."""
    lib().oracle_set_threads(int(n))
