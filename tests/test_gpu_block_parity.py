"""Forces inside real block steps at the sizes of the larger runs: after a
sampled block step, the stored acceleration and jerk of the particles it
advanced (taken at the predicted positions of every particle) against the
oracle fed the same predicted state — every particle predicted from the
previous state over its own interval to the step's time.  Covers the step
path's own plans, records and kernels on partial active sets, both below
and above the size at which the step builds its j records, and the mixed
path's FP64 evaluation of small steps."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import FP64_TOL, check_parity, is_mixed, require_gpu, to_np

pytestmark = pytest.mark.gpu

TICK = 2.0 ** -20
SMALL_STEP = 256      # mixed block steps with at most this many active run in FP64,
SMALL_WORK = 1 << 27  # and so do those of at most this many interactions


def _state(g):
    return {k: to_np(t) for k, t in g.get_state().items()}


def _check_block_steps(g, m, eps, t_end, checks, every, sample, mixed, label):
    rng = np.random.default_rng(17)
    n = m.shape[0]
    sizes = []
    for c in range(checks):
        if every > 1:
            g.step_blocks(t_end, every - 1)
        s0 = _state(g)
        ns, _ = g.step_blocks(t_end, 1)
        assert ns == 1
        s1 = _state(g)
        active = np.nonzero(s1["tick"] != s0["tick"])[0]
        assert active.size > 0
        t_next = s1["tick"][active]
        assert np.all(t_next == t_next[0])
        dt = (t_next[0] - s0["tick"]) * TICK
        xp, vp = oracle.predict(s0["x"], s0["v"], s0["a"], s0["j"], dt)
        idx = active if active.size <= sample else np.sort(rng.choice(active, sample, False))
        a_ref, j_ref = oracle.forces(xp, vp, m, eps, idx=idx.astype(np.int64))
        print(f"  {label} check {c}: n_active {active.size} of {n}", flush=True)
        st = check_parity(s1["a"][idx], s1["j"][idx], a_ref, j_ref, mixed, f"{label} {c}")
        if mixed and (active.size <= SMALL_STEP or active.size * n <= SMALL_WORK):
            # a mixed block step this small is evaluated by the FP64 kernel
            assert st["acc_max"] <= FP64_TOL and st["jerk_max"] <= FP64_TOL, st
        sizes.append(active.size)
    return sizes


def test_fp64_block_steps_plummer_65536():
    # Plummer N = 65536, eps = 1e-3, FP64, levels 2^-6 ... 2^-20
    require_gpu()
    m, x, v = ics.plummer(65536, 2)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, eta=0.01, eta_start=0.01,
                      level_min=6, level_max=20, tuning="auto")
    g.step(1 / 64)
    sizes = _check_block_steps(g, m, 1e-3, 1 / 8, checks=8, every=16, sample=256,
                               mixed=False, label="plummer65536")
    # the next step after a synchronised time moves only the finest level
    assert min(sizes) < 65536 // 16
    g.step(1 / 8)                         # the run still reaches t_end
    assert np.all(_state(g)["tick"] == (1 << 20) // 8)


def test_mixed_block_steps_salpeter_262144():
    # Plummer N = 262144 with Salpeter masses, eps = 1e-4, mixed precision
    require_gpu()
    n = 262144
    m, x, v = ics.plummer(n, 3, masses=ics.salpeter_masses(n, 3))
    g = binding.NBody(m, x, v, eps=1e-4, precision=binding.MIXED, eta=0.01, eta_start=0.01,
                      level_min=7, level_max=20, tuning="auto")
    # the initial evaluation (two passes: jerk estimate, then near pairs)
    s0 = _state(g)
    idx = np.sort(np.random.default_rng(5).choice(n, 8192, False))
    a_ref, j_ref = oracle.forces(x, v, m, 1e-4, idx=idx.astype(np.int64))
    check_parity(s0["a"][idx], s0["j"][idx], a_ref, j_ref, True, "salpeter262144 t=0")
    g.step(1 / 128)
    _check_block_steps(g, m, 1e-4, 1 / 16, checks=8, every=24, sample=8192, mixed=True,
                       label="salpeter262144")


@pytest.mark.parametrize("small_log2,level_max", [(20, 10), (-1, 10), (-1, 20)])
def test_mixed_ensemble_block_steps_both_routes(small_log2, level_max):
    # three clusters in one context, mixed precision.  small_log2 = 20: a
    # step is routed to the FP64 kernel when n_active x N_c <= 2^20 (or at
    # most 256 active), so within one block step the largest cluster runs
    # the mixed kernels while the smallest runs the FP64 one; -1: every
    # step of every cluster runs the mixed kernels.  Each cluster's stored
    # forces after a step against the oracle on that cluster's predicted
    # state.  level_max = 10 holds most particles on the finest level (large
    # active sets); level_max = 20 gives the small sets of the finest levels.
    require_gpu()
    sizes = [12000, 3000, 500]
    m, x, v, off = ics.ensemble(3, sizes=sizes, seed=77)
    eps = [1e-3, 2e-3, 1e-3]
    g = binding.NBody(m, x, v, eps=eps, cluster_offsets=off, precision=binding.MIXED,
                      eta=0.01, eta_start=0.01, level_min=4, level_max=level_max,
                      tuning={"small_log2": small_log2})
    rng = np.random.default_rng(9)
    seen_mixed = seen_small = False
    st_prev = g.stats()
    for step in range(48):
        s0 = _state(g)
        ns, _ = g.step_blocks(0.25, 1)
        assert ns == 1
        s1 = _state(g)
        st = g.stats()
        d_all = st["interactions"] - st_prev["interactions"]
        d_small = st["small_step_interactions"] - st_prev["small_step_interactions"]
        st_prev = st
        assert 0 <= d_small <= d_all
        if small_log2 < 0:
            assert d_small == 0
        for c in range(3):
            sl = slice(off[c], off[c + 1])
            act = np.nonzero(s1["tick"][sl] != s0["tick"][sl])[0]
            if act.size == 0:
                continue
            nc = sizes[c]
            routed_small = small_log2 >= 0 and (act.size <= 256 or act.size * nc <= 1 << 20)
            seen_small |= routed_small
            seen_mixed |= not routed_small
            t_next = s1["tick"][sl][act]
            assert np.all(t_next == t_next[0])
            dt = (t_next[0] - s0["tick"][sl]) * TICK
            xp, vp = oracle.predict(s0["x"][sl], s0["v"][sl], s0["a"][sl], s0["j"][sl], dt)
            idx = act if act.size <= 512 else np.sort(rng.choice(act, 512, False))
            a_ref, j_ref = oracle.forces(xp, vp, m[sl], eps[c], idx=idx.astype(np.int64))
            a1, j1 = s1["a"][sl][idx], s1["j"][sl][idx]
            st_c = check_parity(a1, j1, a_ref, j_ref, True, f"step {step} cluster {c}")
            if routed_small:
                assert st_c["acc_max"] <= FP64_TOL and st_c["jerk_max"] <= FP64_TOL, st_c
    assert seen_mixed
    if small_log2 >= 0:
        assert seen_small


def test_whole_level_step_builds_records():
    # a block step that moves every particle of a level >= n/16 takes the
    # record path (and the broadcast kernel under the FP64 tuning)
    require_gpu()
    n = 16384
    m, x, v = ics.plummer(n, 8)
    for prec in (binding.FP64, binding.MIXED, binding.MIXED_DS):
        g = binding.NBody(m, x, v, eps=1e-3, precision=prec, dt_shared=1 / 256, level_min=4,
                          level_max=8, tuning={"variant": binding.VARIANT_S2
                                               if prec == binding.FP64 else binding.VARIANT_K1})
        sizes = _check_block_steps(g, m, 1e-3, 1 / 16, checks=2, every=1, sample=512,
                                   mixed=is_mixed(prec), label=f"shared prec={prec}")
        assert sizes == [n, n]
        g.close()
