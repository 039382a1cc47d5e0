"""Parity at the benchmark's full size and launch configuration: King W0=7,
N = 2^20, eps = 1e-4, every particle active (the evaluation nbody_init and
each benchmark block step run).  The oracle computes a bounded random sample
of i one by one against all 2^20 j."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import check_parity, require_gpu, to_np, is_mixed

pytestmark = pytest.mark.gpu

N = 1 << 20
EPS = 1e-4
LEVEL = 10


@pytest.fixture(scope="module")
def king():
    return ics.king(N, 7.0, 4)


@pytest.mark.parametrize("prec", [binding.FP64, binding.MIXED, binding.MIXED_DS])
def test_full_size_sampled(king, prec):
    require_gpu()
    m, x, v = king
    print(f"full size prec={prec}", flush=True)
    # the benchmark's configuration: autotuned launch shapes (applied after
    # the initial evaluation), one block step per launch
    g = binding.NBody(m, x, v, eps=EPS, precision=prec, level_min=LEVEL, level_max=LEVEL,
                      tuning="auto")
    g.set_tuning({"steps_per_launch": 1})
    rng = np.random.default_rng(44)
    idx = np.sort(rng.choice(N, 4096, replace=False)).astype(np.int64)
    # the initial full evaluation (state source, all active)
    s0 = {k: to_np(t) for k, t in g.get_state().items()}
    a_ref, j_ref = oracle.forces(x, v, m, EPS, idx=idx)
    mixed = is_mixed(prec)
    check_parity(s0["a"][idx], s0["j"][idx], a_ref, j_ref, mixed, "t=0")
    # one benchmark block step: forces at the predicted positions
    g.step(2.0 ** -LEVEL)
    s1 = {k: to_np(t) for k, t in g.get_state().items()}
    assert np.all(s1["tick"] == 1 << (20 - LEVEL))
    xp, vp = oracle.predict(x, v, s0["a"], s0["j"], 2.0 ** -LEVEL)
    a_ref, j_ref = oracle.forces(xp, vp, m, EPS, idx=idx)
    check_parity(s1["a"][idx], s1["j"][idx], a_ref, j_ref, mixed, "after one step")
    # momentum balance over all particles (Newton's third law)
    for q in ("a", "j"):
        tot = np.linalg.norm((m[:, None] * s1[q]).sum(axis=0))
        scale = (m[:, None] * np.abs(s1[q])).sum()
        assert tot <= (1e-12 if prec == binding.FP64 else 1e-6) * scale
    g.close()
