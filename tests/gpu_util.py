"""Helpers shared by the GPU tests (comparison metrics, device fixtures)."""
import numpy as np
import pytest

FP64_TOL = 1e-12     # plain FP64 GPU path vs the oracle, per-particle relative
MIXED_TOL = 1e-6     # mixed-precision path vs the oracle


def rel_err(got, ref):
    """Per-particle relative error |got - ref| / |ref| (absolute where |ref| = 0)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0909_0879_amd import binding
    binding.lib()      # raises if the HIP library is missing: no fallback
    return torch


def to_np(t):
    return t.detach().cpu().numpy()
