"""Helpers shared by the GPU tests (comparison metrics, device fixtures)."""
import numpy as np
import pytest

FP64_TOL = 1e-12     # plain FP64 GPU path vs the oracle, per-particle relative
MIXED_TOL = 1e-6     # mixed paths: acceleration and jerk, max over particles


def is_mixed(prec):
    """FP32 pair arithmetic (either mixed form): the mixed tolerances apply."""
    from paper_0909_0879_amd import binding
    return prec in (binding.MIXED, binding.MIXED_DS)


def rel_err(got, ref):
    """Per-particle relative error |got - ref| / |ref| (absolute where |ref| = 0)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def check_parity(acc, jerk, a_ref, j_ref, mixed, label=""):
    """Assert the parity bar for one path and return the error stats."""
    ea, ej = rel_err(acc, a_ref), rel_err(jerk, j_ref)
    st = {"acc_max": float(ea.max()), "acc_med": float(np.median(ea)),
          "jerk_max": float(ej.max()), "jerk_med": float(np.median(ej))}
    print(f"  parity {label} {st}", flush=True)
    if mixed:
        assert st["acc_max"] <= MIXED_TOL, st
        assert st["jerk_max"] <= MIXED_TOL, st
    else:
        assert st["acc_max"] <= FP64_TOL, st
        assert st["jerk_max"] <= FP64_TOL, st
    return st


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0909_0879_amd import binding
    binding.lib()      # raises if the HIP library is missing: no fallback
    return torch


def to_np(t):
    return t.detach().cpu().numpy()
