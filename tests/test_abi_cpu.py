"""C ABI checks that need no GPU: the library loads, exports every function
include/nbody.h declares, and rejects bad arguments on the host before any
device call (or reports a missing device)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_0909_0879_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    decl = declared_functions()
    assert len(decl) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (nbody_\w+)", out))
    for name in decl:
        assert name in exported, name
        getattr(lib, name)
    assert sorted(binding.EXPORTED) == sorted(decl)


def test_strerror_codes():
    lib = binding.lib()
    for code in range(0, -8, -1):
        s = lib.nbody_strerror(code).decode()
        assert s and s != "unknown error"
    assert lib.nbody_strerror(-99).decode() == "unknown error"


def _params(n=16, **kw):
    return binding.make_params(n, **kw)


def test_workspace_bytes_host_only():
    b1 = binding.workspace_bytes(1024)
    b2 = binding.workspace_bytes(2048)
    assert 0 < b1 < b2
    assert b1 % 256 == 0
    # ensemble needs per-cluster tables
    off = np.arange(0, 1025, 2, dtype=np.int64)
    assert binding.workspace_bytes(1024, n_clusters=512, cluster_offsets=off, eps=[1e-3] * 512) > b1


def test_precisions_accepted_and_workspace_holds_the_split_rows():
    lib = binding.lib()
    for prec in (binding.FP64, binding.MIXED, binding.MIXED_DS):
        p = _params(precision=prec)
        assert lib.nbody_workspace_bytes(C.byref(p), 16) > 0, prec
    p = _params(precision=3)
    assert lib.nbody_workspace_bytes(C.byref(p), 16) == 0
    # the planner gives a cluster up to 32 partial rows (8 doubles each) per
    # j-particle, so the workspace must hold 32 n rows besides the state
    for n in (1 << 10, 1 << 16, 1 << 20):
        assert binding.workspace_bytes(n) >= 32 * 8 * 8 * n, n


@pytest.mark.parametrize("bad", [
    dict(eps=-1.0), dict(eps=float("nan")), dict(eta=0.0), dict(eta_start=-1.0),
    dict(level_min=5, level_max=4), dict(level_max=21), dict(level_min=-1),
    dict(dt_shared=0.3), dict(dt_shared=2.0 ** -9, level_min=3, level_max=8),
    dict(precision=7),
])
def test_invalid_params_rejected_on_host(bad):
    lib = binding.lib()
    p = _params(**bad)
    assert lib.nbody_workspace_bytes(C.byref(p), 16) == 0
    ctx = C.c_void_p()
    fake = C.c_void_p(0x1000)
    p.workspace = 0x100000
    p.workspace_bytes = 1 << 40
    rc = lib.nbody_init(C.byref(ctx), C.byref(p), 16, fake, fake, fake)
    assert rc == binding.EINVAL
    assert ctx.value is None
    assert lib.nbody_last_error().decode()


def test_field_parameters_checked_on_host():
    lib = binding.lib()
    good = binding.allen_santillan()
    p = _params(field=good)
    assert lib.nbody_workspace_bytes(C.byref(p), 16) > 0
    # scaling to other units keeps the model's dimensionless shape
    f = binding.allen_santillan(length_unit_kpc=1e-3, mass_unit_msun=1e5)
    assert f["halo_gamma"] == good["halo_gamma"]
    assert f["disk_a"] / f["disk_b"] == good["disk_a"] / good["disk_b"]
    assert abs(f["bulge_m"] / good["bulge_m"] - 2.32e7 / 1e5) < 1e-9
    for bad in (dict(disk_b=0.0), dict(bulge_b=0.0), dict(halo_a=0.0), dict(halo_rc=-1.0),
                dict(halo_gamma=0.0), dict(disk_a=-1.0), dict(bulge_m=-1.0),
                dict(halo_m=float("nan")), dict(disk_a=float("inf"))):
        p = _params(field={**good, **bad})
        assert lib.nbody_workspace_bytes(C.byref(p), 16) == 0, bad
    # a switched-off component needs no valid scales
    p = _params(field={"bulge_m": 0.0, "bulge_b": 0.0, "halo_m": 1.0, "halo_a": 2.0,
                       "halo_gamma": 1.0, "halo_rc": 10.0})
    assert lib.nbody_workspace_bytes(C.byref(p), 16) > 0
    try:
        binding.make_params(16, field={"bulge_mass": 1.0})
        raise AssertionError("unknown key accepted")
    except ValueError:
        pass


def test_bad_cluster_offsets_rejected():
    lib = binding.lib()
    for off in ([0, 10, 10, 16], [1, 10, 16], [0, 10, 15]):
        p = _params(16, n_clusters=len(off) - 1, cluster_offsets=off, eps=[1e-3] * (len(off) - 1))
        assert lib.nbody_workspace_bytes(C.byref(p), 16) == 0


def test_init_argument_checks_before_device():
    lib = binding.lib()
    p = _params()
    need = lib.nbody_workspace_bytes(C.byref(p), 16)
    ctx = C.c_void_p()
    fake = C.c_void_p(0x1000)
    # NULL arrays
    p.workspace, p.workspace_bytes = 0x100000, need
    assert lib.nbody_init(C.byref(ctx), C.byref(p), 16, None, fake, fake) == binding.EINVAL
    # misaligned workspace
    p.workspace = 0x100010
    assert lib.nbody_init(C.byref(ctx), C.byref(p), 16, fake, fake, fake) == binding.EINVAL
    # too small
    p.workspace, p.workspace_bytes = 0x100000, need - 256
    assert lib.nbody_init(C.byref(ctx), C.byref(p), 16, fake, fake, fake) == binding.ENOMEM
    # n out of range
    p.workspace_bytes = need
    assert lib.nbody_init(C.byref(ctx), C.byref(p), 0, fake, fake, fake) == binding.EINVAL


def test_no_device_reported(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = binding.lib()
    p = _params()
    need = lib.nbody_workspace_bytes(C.byref(p), 16)
    p.workspace, p.workspace_bytes = 0x100000, need
    ctx = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert lib.nbody_init(C.byref(ctx), C.byref(p), 16, fake, fake, fake) == binding.ENODEV


def test_null_context_calls():
    lib = binding.lib()
    fake = C.c_void_p(0x1000)
    assert lib.nbody_forces(None, fake, 1, fake, fake, fake, 1, fake, fake) == binding.EINVAL
    assert lib.nbody_step(None, 1.0, None, None) == binding.EINVAL
    assert lib.nbody_energy(None, fake) == binding.EINVAL
    assert lib.nbody_sync(None) == binding.EINVAL
    assert lib.nbody_accel(None, fake, 1, fake, fake, 1, fake) == binding.EINVAL
    assert lib.nbody_step_symplectic(None, binding.LEAPFROG, 1 / 64, 4, None) == binding.EINVAL
    assert lib.nbody_step_blocks(None, 1.0, 1, None, None) == binding.EINVAL
    assert lib.nbody_get_state(None, fake, fake, fake, fake, fake, fake) == binding.EINVAL
    assert lib.nbody_set_state(None, fake, fake, fake, fake, fake, fake) == binding.EINVAL
    lib.nbody_destroy(None)


def test_tuning_struct_roundtrip():
    t = binding.Tuning.from_dict({"variant": 2, "i_slots": [1] * 25, "target_items": [64] * 25})
    assert t.as_dict()["i_slots"][3] == 1
    assert C.sizeof(binding.Tuning) == 4 * (8 + 2 * binding.TUNE_BUCKETS)


def test_noalloc_limits_checked_on_host():
    # sizes beyond the fixed scratch and bad arguments are rejected before
    # any device work (no GPU needed)
    lib = binding.lib()
    fake = C.c_void_p(0x1000)
    f = lib.nbody_forces_noalloc
    assert f(binding.MIXED, 1e-3, fake, 10, fake, fake, fake, 16385, fake, fake, None) == binding.EINVAL
    assert f(binding.MIXED, 1e-3, fake, 16385, fake, fake, fake, 100, fake, fake, None) == binding.EINVAL
    assert f(3, 1e-3, fake, 10, fake, fake, fake, 100, fake, fake, None) == binding.EINVAL
    assert f(binding.FP64, -1.0, fake, 10, fake, fake, fake, 100, fake, fake, None) == binding.EINVAL
    assert f(binding.FP64, 1e-3, None, 10, fake, fake, fake, 100, fake, fake, None) == binding.EINVAL
    assert f(binding.FP64, 1e-3, fake, 0, fake, fake, fake, 100, fake, fake, None) == binding.OK
