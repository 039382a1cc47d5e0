"""Thin ctypes binding of libnbody.so (argument marshalling only).

Every step of the hot path runs in the HIP library; this module only turns
torch device tensors into pointers, holds the workspace tensor and maps
error codes to exceptions.  PyTorch is used for device memory and streams.
If the compiled library is missing the import fails: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")

OK, EINVAL, ENODEV, ENOMEM, EHIP, EINDEX, ENONFINITE, EDOMAIN = 0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED, MIXED_DS = 0, 1, 2   # nbody_precision
VARIANT_DEFAULT, VARIANT_K1, VARIANT_K2, VARIANT_S1, VARIANT_S2 = 0, 1, 2, 3, 4
GRAPH_ON, GRAPH_OFF = 1, 2
LEAPFROG, SYMPLECTIC6 = 0, 1
TUNE_BUCKETS = 25
TICK_BITS = 20

EXPORTED = [
    "nbody_workspace_bytes", "nbody_init", "nbody_forces", "nbody_step", "nbody_energy",
    "nbody_get_state", "nbody_set_state", "nbody_sync", "nbody_stats", "nbody_destroy",
    "nbody_strerror", "nbody_last_error", "nbody_get_tuning", "nbody_set_tuning",
    "nbody_profile", "nbody_profile_read", "nbody_accel", "nbody_step_symplectic",
    "nbody_step_blocks", "nbody_forces_noalloc",
]


class NBodyError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


FIELD_KEYS = ("bulge_m", "bulge_b", "disk_m", "disk_a", "disk_b", "halo_m", "halo_a",
              "halo_gamma", "halo_rc")


class Field(C.Structure):
    """nbody_field: the external Galactic field (G = 1, context units)."""
    _fields_ = [(k, C.c_double) for k in FIELD_KEYS]


class Params(C.Structure):
    _fields_ = [
        ("n_clusters", C.c_int32), ("precision", C.c_int32),
        ("cluster_offsets", C.c_void_p), ("eps", C.c_void_p),
        ("eta", C.c_double), ("eta_start", C.c_double), ("dt_shared", C.c_double),
        ("level_min", C.c_int32), ("level_max", C.c_int32),
        ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("field", C.POINTER(Field)),
    ]


# The Galactic model of Allen & Santillan (1991) in its own units (1 kpc,
# 2.32e7 M_sun, G = 1), the external field the paper adds (Sect. 4).
ALLEN_SANTILLAN_1991 = {"bulge_m": 606.0, "bulge_b": 0.3873,
                        "disk_m": 3690.0, "disk_a": 5.3178, "disk_b": 0.25,
                        "halo_m": 4615.0, "halo_a": 12.0, "halo_gamma": 1.02,
                        "halo_rc": 100.0}
AS91_MASS_UNIT_MSUN = 2.32e7


def allen_santillan(length_unit_kpc: float = 1.0, mass_unit_msun: float = AS91_MASS_UNIT_MSUN):
    """The Allen & Santillan field in units where the length unit is
    length_unit_kpc and the mass unit mass_unit_msun (G = 1 in both)."""
    out = {}
    for k, val in ALLEN_SANTILLAN_1991.items():
        if k.endswith("_m"):
            out[k] = val * AS91_MASS_UNIT_MSUN / mass_unit_msun
        elif k == "halo_gamma":
            out[k] = val
        else:
            out[k] = val / length_unit_kpc
    return out


class Tuning(C.Structure):
    _fields_ = [
        ("variant", C.c_int32), ("use_graph", C.c_int32), ("steps_per_launch", C.c_int32),
        ("min_split_j", C.c_int32), ("refine_ratio", C.c_float),
        ("i_slots", C.c_int32 * TUNE_BUCKETS), ("target_items", C.c_int32 * TUNE_BUCKETS),
        ("acc_variant", C.c_int32), ("near_jerk", C.c_float), ("small_log2", C.c_int32),
    ]

    def as_dict(self):
        return {"variant": self.variant, "use_graph": self.use_graph,
                "steps_per_launch": self.steps_per_launch, "min_split_j": self.min_split_j,
                "refine_ratio": self.refine_ratio,
                "i_slots": list(self.i_slots), "target_items": list(self.target_items),
                "acc_variant": self.acc_variant, "near_jerk": self.near_jerk,
                "small_log2": self.small_log2}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.variant = int(d.get("variant", 0))
        t.use_graph = int(d.get("use_graph", 0))
        t.steps_per_launch = int(d.get("steps_per_launch", 0))
        t.min_split_j = int(d.get("min_split_j", 0))
        t.refine_ratio = float(d.get("refine_ratio", 0.0))
        for b, v in enumerate(d.get("i_slots", [0] * TUNE_BUCKETS)):
            t.i_slots[b] = int(v)
        for b, v in enumerate(d.get("target_items", [0] * TUNE_BUCKETS)):
            t.target_items[b] = int(v)
        t.acc_variant = int(d.get("acc_variant", 0))
        t.near_jerk = float(d.get("near_jerk", 0.0))
        t.small_log2 = int(d.get("small_log2", 0))
        return t


_lib = None


def lib():
    """Load libnbody.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_0909_0879_amd/build_lib.py")
        L = C.CDLL(LIB_PATH)
        P, I64 = C.c_void_p, C.c_int64
        L.nbody_workspace_bytes.argtypes = [P, I64]
        L.nbody_workspace_bytes.restype = C.c_size_t
        L.nbody_init.argtypes = [P, P, I64, P, P, P]
        L.nbody_forces.argtypes = [P, P, I64, P, P, P, I64, P, P]
        L.nbody_step.argtypes = [P, C.c_double, P, P]
        L.nbody_energy.argtypes = [P, P]
        L.nbody_get_state.argtypes = [P, P, P, P, P, P, P]
        L.nbody_set_state.argtypes = [P, P, P, P, P, P, P]
        L.nbody_sync.argtypes = [P]
        L.nbody_stats.argtypes = [P, P]
        L.nbody_destroy.argtypes = [P]
        L.nbody_destroy.restype = None
        L.nbody_strerror.argtypes = [C.c_int]
        L.nbody_strerror.restype = C.c_char_p
        L.nbody_last_error.argtypes = []
        L.nbody_last_error.restype = C.c_char_p
        L.nbody_get_tuning.argtypes = [P, P]
        L.nbody_set_tuning.argtypes = [P, P]
        L.nbody_profile.argtypes = [P, C.c_int]
        L.nbody_profile_read.argtypes = [P, P, P, P, P]
        L.nbody_accel.argtypes = [P, P, C.c_int64, P, P, C.c_int64, P]
        L.nbody_step_symplectic.argtypes = [P, C.c_int, C.c_double, C.c_int64, P]
        L.nbody_step_blocks.argtypes = [P, C.c_double, C.c_int64, P, P]
        L.nbody_forces_noalloc.argtypes = [C.c_int, C.c_double, P, I64, P, P, P, I64, P, P, P]
        _lib = L
    return _lib


def check(rc: int, where: str):
    if rc != OK:
        msg = lib().nbody_last_error().decode() or lib().nbody_strerror(rc).decode()
        raise NBodyError(rc, where, msg)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream), stream


def make_params(n, n_clusters=1, cluster_offsets=None, eps=1e-3, precision=FP64, eta=0.01,
                eta_start=0.01, dt_shared=0.0, level_min=3, level_max=20, field=None):
    """Host-side parameter block (keeps the numpy arrays it points to alive).
    field: dict of FIELD_KEYS (missing components off) or None."""
    eps_arr = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float64), (n_clusters,)))
    p = Params()
    p.n_clusters = n_clusters
    p.precision = precision
    keep = [eps_arr]
    if cluster_offsets is not None:
        off = np.ascontiguousarray(cluster_offsets, np.int64)
        keep.append(off)
        p.cluster_offsets = off.ctypes.data
    else:
        p.cluster_offsets = None
    p.eps = eps_arr.ctypes.data
    p.eta, p.eta_start, p.dt_shared = float(eta), float(eta_start), float(dt_shared)
    p.level_min, p.level_max = int(level_min), int(level_max)
    if field is not None:
        unknown = set(field) - set(FIELD_KEYS)
        if unknown:
            raise ValueError(f"unknown field keys {sorted(unknown)}")
        f = Field(*[float(field.get(k, 0.0)) for k in FIELD_KEYS])
        keep.append(f)
        p.field = C.pointer(f)
    p._keep = keep
    return p


def workspace_bytes(n, **kw) -> int:
    p = make_params(n, **kw)
    return int(lib().nbody_workspace_bytes(C.byref(p), int(n)))


def nbody_forces_noalloc(precision, eps, i_active, xj, vj, mj, acc, jerk, stream=None):
    """nbody_forces_noalloc on device tensors the caller provides (i_active
    int32 (n_active,), xj, vj (n_j, 3), mj (n_j,), acc, jerk (n_active, 3),
    all float64 and contiguous; jerk may be None): the one-cluster
    evaluation that allocates nothing, enqueued on `stream` (default: the
    current stream).  Marshalling only."""
    handle, _ = _stream_handle(stream)
    na = int(i_active.shape[0])
    nj = int(mj.shape[0])
    check(lib().nbody_forces_noalloc(int(precision), float(eps), _ptr(i_active), na, _ptr(xj),
                                     _ptr(vj), _ptr(mj), nj, _ptr(acc), _ptr(jerk), handle),
          "nbody_forces_noalloc")


class NBody:
    """One library context: state in a caller-owned torch workspace tensor."""

    def __init__(self, m, x, v, *, cluster_offsets=None, eps=1e-3, precision=FP64, eta=0.01,
                 eta_start=0.01, dt_shared=0.0, level_min=3, level_max=20, stream=None,
                 device="cuda", tuning=None, field=None):
        import torch
        self._torch = torch
        m = torch.as_tensor(m, dtype=torch.float64, device=device).contiguous()
        x = torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
        v = torch.as_tensor(v, dtype=torch.float64, device=device).contiguous()
        n = m.shape[0]
        if x.shape != (n, 3) or v.shape != (n, 3):
            raise ValueError("x and v must have shape (n, 3)")
        n_clusters = 1 if cluster_offsets is None else len(cluster_offsets) - 1
        self.params = make_params(n, n_clusters, cluster_offsets, eps, precision, eta, eta_start,
                                  dt_shared, level_min, level_max, field)
        self.n = n
        self.n_clusters = n_clusters
        self.precision = precision
        self.level_min, self.level_max = level_min, level_max
        nbytes = lib().nbody_workspace_bytes(C.byref(self.params), n)
        if nbytes == 0:
            check(EINVAL, "nbody_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h, self.stream = _stream_handle(stream)
        self.params.stream = h
        self.params.workspace = self.workspace.data_ptr()
        self.params.workspace_bytes = nbytes
        self.ctx = C.c_void_p()
        check(lib().nbody_init(C.byref(self.ctx), C.byref(self.params), n, _ptr(m), _ptr(x),
                               _ptr(v)), "nbody_init")
        if tuning == "auto":
            from . import autotune
            tuning = autotune.load(precision, n, n_clusters=n_clusters)
        if tuning:
            self.set_tuning(tuning)

    # -- evaluation -------------------------------------------------------
    def forces(self, xj, vj, mj, i_active=None):
        """Acceleration and jerk on i_active from (xj, vj, mj); device tensors."""
        torch = self._torch
        dev = self.workspace.device
        xj = torch.as_tensor(xj, dtype=torch.float64, device=dev).contiguous()
        vj = torch.as_tensor(vj, dtype=torch.float64, device=dev).contiguous()
        mj = torch.as_tensor(mj, dtype=torch.float64, device=dev).contiguous()
        nj = mj.shape[0]
        if i_active is None:
            i_active = torch.arange(nj, dtype=torch.int32, device=dev)
        ia = torch.as_tensor(i_active, dtype=torch.int32, device=dev).contiguous()
        na = ia.shape[0]
        acc = torch.empty((na, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty((na, 3), dtype=torch.float64, device=dev)
        check(lib().nbody_forces(self.ctx, _ptr(ia), na, _ptr(xj), _ptr(vj), _ptr(mj), nj,
                                 _ptr(acc), _ptr(jerk)), "nbody_forces")
        return acc, jerk

    def accel(self, xj, mj, i_active=None):
        """Acceleration only on i_active from (xj, mj); device tensors."""
        torch = self._torch
        dev = self.workspace.device
        xj = torch.as_tensor(xj, dtype=torch.float64, device=dev).contiguous()
        mj = torch.as_tensor(mj, dtype=torch.float64, device=dev).contiguous()
        nj = mj.shape[0]
        if i_active is None:
            i_active = torch.arange(nj, dtype=torch.int32, device=dev)
        ia = torch.as_tensor(i_active, dtype=torch.int32, device=dev).contiguous()
        na = ia.shape[0]
        acc = torch.empty((na, 3), dtype=torch.float64, device=dev)
        check(lib().nbody_accel(self.ctx, _ptr(ia), na, _ptr(xj), _ptr(mj), nj, _ptr(acc)),
              "nbody_accel")
        return acc

    def step_symplectic(self, scheme, h, n_steps):
        """n_steps steps of size h with LEAPFROG or SYMPLECTIC6; returns the
        pair slots evaluated."""
        ni = C.c_int64(0)
        check(lib().nbody_step_symplectic(self.ctx, int(scheme), float(h), int(n_steps),
                                          C.byref(ni)), "nbody_step_symplectic")
        return ni.value

    def step(self, t_end):
        ns, ni = C.c_int64(0), C.c_int64(0)
        check(lib().nbody_step(self.ctx, float(t_end), C.byref(ns), C.byref(ni)), "nbody_step")
        return ns.value, ni.value

    def step_blocks(self, t_end, max_block_steps):
        """At most max_block_steps block steps toward t_end."""
        ns, ni = C.c_int64(0), C.c_int64(0)
        check(lib().nbody_step_blocks(self.ctx, float(t_end), int(max_block_steps), C.byref(ns),
                                      C.byref(ni)), "nbody_step_blocks")
        return ns.value, ni.value

    def energy(self):
        out = np.empty((self.n_clusters, 9))
        check(lib().nbody_energy(self.ctx, out.ctypes.data_as(C.c_void_p)), "nbody_energy")
        return out

    def get_state(self):
        torch = self._torch
        dev = self.workspace.device
        x, v, a, j = (torch.empty((self.n, 3), dtype=torch.float64, device=dev) for _ in range(4))
        tick = torch.empty(self.n, dtype=torch.int64, device=dev)
        level = torch.empty(self.n, dtype=torch.int8, device=dev)
        check(lib().nbody_get_state(self.ctx, _ptr(x), _ptr(v), _ptr(a), _ptr(j), _ptr(tick),
                                    _ptr(level)), "nbody_get_state")
        return {"x": x, "v": v, "a": a, "j": j, "tick": tick, "level": level}

    def set_state(self, st):
        torch = self._torch
        dev = self.workspace.device
        f = lambda k: torch.as_tensor(st[k], dtype=torch.float64, device=dev).contiguous()
        x, v, a, j = f("x"), f("v"), f("a"), f("j")
        tick = torch.as_tensor(st["tick"], dtype=torch.int64, device=dev).contiguous()
        level = torch.as_tensor(st["level"], dtype=torch.int8, device=dev).contiguous()
        check(lib().nbody_set_state(self.ctx, _ptr(x), _ptr(v), _ptr(a), _ptr(j), _ptr(tick),
                                    _ptr(level)), "nbody_set_state")

    def sync(self):
        check(lib().nbody_sync(self.ctx), "nbody_sync")

    def stats(self):
        out = np.zeros(8, np.int64)
        check(lib().nbody_stats(self.ctx, out.ctypes.data_as(C.c_void_p)), "nbody_stats")
        return {"block_steps": int(out[0]), "interactions": int(out[1]),
                "floor_clamps": int(out[2]), "t_tick": int(out[3]), "refined": int(out[4]),
                "near_pairs": int(out[5]), "small_step_interactions": int(out[6])}

    def get_tuning(self) -> dict:
        t = Tuning()
        check(lib().nbody_get_tuning(self.ctx, C.byref(t)), "nbody_get_tuning")
        return t.as_dict()

    def set_tuning(self, d: dict):
        t = Tuning.from_dict(d)
        check(lib().nbody_set_tuning(self.ctx, C.byref(t)), "nbody_set_tuning")

    def profile(self, enable: bool):
        check(lib().nbody_profile(self.ctx, 1 if enable else 0), "nbody_profile")

    def profile_read(self):
        """Force-kernel event time since the last read: (ms, launches) of the
        context's own kernel and (ms, launches) of the FP64 re-evaluation."""
        ms, nl, rms, rnl = C.c_double(0.0), C.c_int64(0), C.c_double(0.0), C.c_int64(0)
        check(lib().nbody_profile_read(self.ctx, C.byref(ms), C.byref(nl), C.byref(rms),
                                       C.byref(rnl)), "nbody_profile_read")
        return ms.value, nl.value, rms.value, rnl.value

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().nbody_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
