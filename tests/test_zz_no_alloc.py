"""The evaluation that allocates nothing (nbody_forces_noalloc, for callers
that cannot allocate) against the context's nbody_forces and the oracle:
two calls in a row on the same GPU, the second with a smaller input."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import FP64_TOL, MIXED_TOL, is_mixed, rel_err, require_gpu, to_np

pytestmark = pytest.mark.gpu

PRECS = [binding.FP64, binding.MIXED, binding.MIXED_DS]


def _noalloc(torch, prec, eps, x, v, m, idx):
    dev = torch.device("cuda")
    xt = torch.as_tensor(x, dtype=torch.float64, device=dev).contiguous()
    vt = torch.as_tensor(v, dtype=torch.float64, device=dev).contiguous()
    mt = torch.as_tensor(m, dtype=torch.float64, device=dev).contiguous()
    it = torch.as_tensor(idx, dtype=torch.int32, device=dev).contiguous()
    acc = torch.zeros((len(idx), 3), dtype=torch.float64, device=dev)
    jerk = torch.zeros((len(idx), 3), dtype=torch.float64, device=dev)
    binding.nbody_forces_noalloc(prec, eps, it, xt, vt, mt, acc, jerk)
    torch.cuda.synchronize()
    return to_np(acc), to_np(jerk)


@pytest.mark.parametrize("prec", PRECS)
def test_noalloc_matches_forces_twice_then_smaller(prec):
    torch = require_gpu()
    tol = MIXED_TOL if is_mixed(prec) else FP64_TOL
    rng = np.random.default_rng(314)
    cases = []
    # first call: 6000 particles, all active; second: 1500 particles, a
    # subset with repeats (the array keeps the first call's contents)
    m1, x1, v1 = ics.plummer(6000, 315)
    cases.append((m1, x1, v1, np.arange(6000, dtype=np.int32), 1e-3))
    m2, x2, v2 = ics.plummer(1500, 316)
    m2 = ics.salpeter_masses(1500, 317)
    cases.append((m2, x2, v2, rng.integers(0, 1500, 700).astype(np.int32), 1e-4))
    for m, x, v, idx, eps in cases:
        a, j = _noalloc(torch, prec, eps, x, v, m, idx)
        g = binding.NBody(m, x, v, eps=eps, precision=prec)
        a_ctx, j_ctx = (to_np(t) for t in g.forces(x, v, m, i_active=idx))
        g.sync()
        g.close()
        a_ref, j_ref = oracle.forces(x, v, m, eps, idx=idx)
        print(f"  noalloc prec={prec} n={len(m)} na={len(idx)}: acc {rel_err(a, a_ref).max():.2e} "
              f"jerk {rel_err(j, j_ref).max():.2e}", flush=True)
        assert rel_err(a, a_ref).max() <= tol and rel_err(j, j_ref).max() <= tol
        assert rel_err(a, a_ctx).max() <= 2 * tol and rel_err(j, j_ctx).max() <= 2 * tol
        if prec == binding.FP64:
            # the FP64 path sums the same terms in the same tiles
            assert rel_err(a, a_ctx).max() <= 1e-13


def test_noalloc_largest_size_and_rejects_beyond():
    torch = require_gpu()
    n = 16384
    m, x, v = ics.plummer(n, 318)
    idx = np.arange(0, n, 7, dtype=np.int32)
    a, j = _noalloc(torch, binding.MIXED, 1e-3, x, v, m, idx)
    a_ref, j_ref = oracle.forces(x, v, m, 1e-3, idx=idx)
    assert rel_err(a, a_ref).max() <= MIXED_TOL and rel_err(j, j_ref).max() <= MIXED_TOL
    m2, x2, v2 = ics.plummer(n + 1, 319)
    with pytest.raises(binding.NBodyError) as e:
        _noalloc(torch, binding.MIXED, 1e-3, x2, v2, m2, np.arange(10, dtype=np.int32))
    assert e.value.code == binding.EINVAL
