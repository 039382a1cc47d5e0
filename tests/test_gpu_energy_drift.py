"""Energy drift of the FP64 block-step path against the oracle's (the paper's
energy-conservation check of Sect. 4.1, on the Plummer N = 65536 block-step
workload).  Over a short horizon both runs follow nearly the same
trajectory, so the GPU's relative energy error should be that of the oracle
to well within a factor 2; and halving eta should cut it, as it does for
the fourth-order Hermite scheme on the CPU."""
import time

import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

N = 65536
EPS = 1e-3


def _gpu_drift(m, x, v, eta, t_end, offsets=None):
    g = binding.NBody(m, x, v, eps=EPS, precision=binding.FP64, eta=eta, eta_start=eta,
                      level_min=6, level_max=20, cluster_offsets=offsets, tuning="auto")
    e0 = g.energy()
    g.step(t_end)
    e1 = g.energy()
    g.close()
    return np.abs(e1[:, 2] - e0[:, 2]) / np.abs(e0[:, 2])


def test_fp64_drift_within_2x_of_oracle():
    require_gpu()
    m, x, v = ics.plummer(N, 2)
    t_end = 1 / 64
    d_gpu = float(_gpu_drift(m, x, v, 0.01, t_end)[0])
    ref = oracle.System(m, x, v, EPS, eta=0.01, eta_start=0.01, level_min=6, level_max=20)
    e0 = ref.energy()["E"]
    # t_end is one step of the coarsest level, so the oracle runs it in one
    # call (about a minute on 16 cores)
    print(f"  gpu |dE/E| {d_gpu:.3e}; oracle run to t = {t_end}", flush=True)
    t0 = time.perf_counter()
    ref.run(t_end)
    print(f"  oracle done after {time.perf_counter() - t0:.1f} s", flush=True)
    d_ref = abs(ref.energy()["E"] - e0) / abs(e0)
    print(f"  |dE/E| gpu {d_gpu:.3e} oracle {d_ref:.3e}", flush=True)
    assert d_gpu <= 2 * d_ref and d_ref <= 2 * d_gpu, (d_gpu, d_ref)


def test_fp64_drift_shrinks_with_eta():
    # the Plummer N = 65536 run itself, and the sum over four independent
    # N = 16384 spheres in one batched context (close encounters make a
    # single run's error noisy; fourth order predicts a factor of about 16)
    require_gpu()
    m, x, v = ics.plummer(N, 2)
    mo, xo, vo, off = ics.ensemble(4, sizes=[16384] * 4, seed=31)
    single, batch = {}, {}
    for eta in (0.02, 0.01):
        single[eta] = float(_gpu_drift(m, x, v, eta, 1 / 32)[0])
        batch[eta] = float(_gpu_drift(mo, xo, vo, eta, 1 / 32, offsets=off).sum())
        print(f"  eta {eta}: |dE/E| N=65536 {single[eta]:.3e}, "
              f"four N=16384 (sum) {batch[eta]:.3e}", flush=True)
    assert single[0.01] * 2 < single[0.02], single
    assert batch[0.01] * 4 < batch[0.02], batch
