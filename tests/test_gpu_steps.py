"""Hermite-4 block steps on the GPU (scheduler, predictor, corrector, Aarseth
levels, graph replay, ensemble, checkpoint) against the CPU oracle and
against itself."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import FP64_TOL, check_parity, rel_err, require_gpu, to_np

pytestmark = pytest.mark.gpu


def _state_np(g):
    st = g.get_state()
    return {k: to_np(t) for k, t in st.items()}


def test_shared_steps_match_oracle():
    # Plummer N = 1024, eps = 1e-3, shared dt = 1/256: 16 steps to t = 1/16
    require_gpu()
    m, x, v = ics.plummer(1024, 1)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, dt_shared=1 / 256,
                      level_min=4, level_max=8)
    ns, ni = g.step(1 / 16)
    assert ns == 16 and ni == 16 * 1024 * 1024
    s = _state_np(g)
    ref = oracle.System(m, x, v, 1e-3, dt_shared=1 / 256, level_min=4, level_max=8)
    ref.run(1 / 16)
    assert np.all(s["tick"] == 1 << 16)
    assert np.abs(s["x"] - ref.x).max() <= 1e-10 * np.abs(ref.x).max()
    assert np.abs(s["v"] - ref.v).max() <= 1e-10 * np.abs(ref.v).max()
    assert rel_err(s["a"], ref.a).max() <= 1e-9


def test_initial_levels_and_forces_match_oracle():
    require_gpu()
    m, x, v = ics.plummer(2000, 21)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, eta=0.01, eta_start=0.01,
                      level_min=3, level_max=20)
    s = _state_np(g)
    ref = oracle.System(m, x, v, 1e-3, eta=0.01, eta_start=0.01, level_min=3, level_max=20)
    assert rel_err(s["a"], ref.a).max() <= FP64_TOL
    assert rel_err(s["j"], ref.j).max() <= FP64_TOL
    assert np.array_equal(s["level"].astype(np.int64), ref.level.astype(np.int64))
    assert np.all(s["tick"] == 0)


@pytest.mark.parametrize("n,t_end,lmin", [(256, 0.125, 3), (1500, 0.0625, 4)])
def test_block_steps_match_oracle(n, t_end, lmin):
    require_gpu()
    print(f"block steps n={n}", flush=True)
    m, x, v = ics.plummer(n, 30 + n)
    kw = dict(eta=0.02, eta_start=0.01, level_min=lmin, level_max=20)
    g = binding.NBody(m, x, v, eps=1e-2, precision=binding.FP64, **kw)
    ns, ni = g.step(t_end)
    s = _state_np(g)
    ref = oracle.System(m, x, v, 1e-2, **kw)
    ref.run(t_end)
    assert ns == ref.stats.n_block_steps
    assert ni == ref.stats.n_interactions - n * n      # oracle counts its initial evaluation
    assert np.array_equal(s["level"].astype(np.int64), ref.level.astype(np.int64))
    assert np.all(s["tick"] == ref.tick)
    assert np.abs(s["x"] - ref.x).max() <= 1e-9
    assert np.abs(s["v"] - ref.v).max() <= 1e-8
    assert len(np.unique(s["level"])) > 1


def test_block_mode_single_level_equals_shared_bitwise():
    require_gpu()
    m, x, v = ics.plummer(700, 3)
    a = binding.NBody(m, x, v, eps=1e-2, dt_shared=2.0 ** -7, level_min=7, level_max=7)
    b = binding.NBody(m, x, v, eps=1e-2, dt_shared=0.0, level_min=7, level_max=7)
    a.step(2.0 ** -3)
    b.step(2.0 ** -3)
    sa, sb = _state_np(a), _state_np(b)
    for k in ("x", "v", "a", "j", "tick"):
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("prec", [binding.FP64, binding.MIXED, binding.MIXED_DS])
def test_graph_replay_equals_eager_bitwise(prec):
    require_gpu()
    m, x, v = ics.plummer(1200, 8)
    kw = dict(eps=5e-3, precision=prec, eta=0.02, level_min=3, level_max=20)
    a = binding.NBody(m, x, v, **kw)
    b = binding.NBody(m, x, v, **kw)
    b.set_tuning({"use_graph": binding.GRAPH_OFF, "steps_per_launch": 3})
    a.step(0.125)
    b.step(0.125)
    # a second graph launch sequence on the same context
    a.step(0.25)
    b.step(0.25)
    sa, sb = _state_np(a), _state_np(b)
    for k in ("x", "v", "a", "j", "tick", "level"):
        assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("prec,small_log2", [(binding.FP64, 0), (binding.MIXED, 0),
                                              (binding.MIXED_DS, 0), (binding.MIXED, -1),
                                              (binding.MIXED_DS, -1)])
def test_ensemble_equals_solo_bitwise(prec, small_log2):
    # small_log2 = -1: no block step is routed to the FP64 kernel, so every
    # step of every cluster runs the mixed kernels (records, near pairs,
    # FP64 re-evaluation) inside the batched launches
    require_gpu()
    sizes = [300, 1024, 64, 777]
    m, x, v, off = ics.ensemble(4, sizes=sizes, seed=5000)
    eps = [1e-3, 2e-3, 1e-3, 4e-3]
    kw = dict(precision=prec, eta=0.02, level_min=3, level_max=20)
    tune = {"small_log2": small_log2}
    e = binding.NBody(m, x, v, eps=eps, cluster_offsets=off, tuning=tune, **kw)
    e.step(0.125)
    st = e.stats()
    if small_log2 < 0:
        assert st["small_step_interactions"] == 0, st
    elif prec != binding.FP64:
        # clusters this small take every block step in FP64 by default
        assert st["small_step_interactions"] == st["interactions"], st
    se = _state_np(e)
    energies = e.energy()
    refined_solo = 0
    for c in range(4):
        sl = slice(off[c], off[c + 1])
        s = binding.NBody(m[sl], x[sl], v[sl], eps=eps[c], tuning=tune, **kw)
        s.step(0.125)
        refined_solo += s.stats()["refined"]
        ss = _state_np(s)
        for k in ("x", "v", "a", "j", "tick", "level"):
            assert np.array_equal(se[k][sl], ss[k]), (c, k)
        es = s.energy()[0]
        assert np.allclose(energies[c], es, rtol=0, atol=1e-15)
    if small_log2 < 0:
        # the FP64 re-evaluation ran, and a cluster alone (whose flagged
        # entries are appended in any order) re-evaluates exactly the
        # particles it re-evaluates inside the ensemble (ordered list)
        assert st["refined"] > 0, st
        assert refined_solo == st["refined"], (refined_solo, st["refined"])


def test_checkpoint_resume_bitwise():
    require_gpu()
    m, x, v = ics.plummer(900, 12)
    kw = dict(eps=2e-3, precision=binding.FP64, eta=0.02, level_min=3, level_max=20)
    a = binding.NBody(m, x, v, **kw)
    a.step(0.125)
    mid = a.get_state()
    a.step(0.25)
    b = binding.NBody(m, x, v, **kw)
    b.set_state(mid)
    b.step(0.25)
    sa, sb = _state_np(a), _state_np(b)
    for k in ("x", "v", "a", "j", "tick", "level"):
        assert np.array_equal(sa[k], sb[k]), k


def test_set_state_validates():
    require_gpu()
    m, x, v = ics.plummer(64, 2)
    g = binding.NBody(m, x, v, eps=1e-3, level_min=3, level_max=20)
    st = g.get_state()
    bad = dict(st)
    bad["tick"] = st["tick"].clone()
    bad["level"] = st["level"].clone()
    bad["level"][0] = 10
    bad["tick"][0] = 3          # not a multiple of 2^10 ticks
    with pytest.raises(binding.NBodyError) as e:
        g.set_state(bad)
    assert e.value.code == binding.EINVAL
    bad["tick"][0] = 0
    bad["level"][0] = 25        # out of range
    with pytest.raises(binding.NBodyError):
        g.set_state(bad)
    g.set_state(st)             # a valid state is accepted again


def test_energy_matches_oracle():
    require_gpu()
    m, x, v = ics.plummer(3000, 17)
    r = oracle.energy(x, v, m, 1e-3)
    for prec in (binding.FP64, binding.MIXED, binding.MIXED_DS):
        g = binding.NBody(m, x, v, eps=1e-3, precision=prec)
        # the context's tuning, then the largest split target (the energy
        # evaluation caps its own splits)
        for tu in (None, {"i_slots": [256] * 25, "target_items": [1 << 20] * 25,
                          "min_split_j": 64}):
            if tu:
                g.set_tuning(tu)
            e = g.energy()[0]
            assert abs(e[0] - r["K"]) <= 1e-14 * abs(r["K"])
            assert abs(e[1] - r["W"]) <= 1e-13 * abs(r["W"])
            assert np.allclose(e[3:6], r["L"], rtol=1e-12, atol=1e-16)
            assert np.allclose(e[6:9], r["P"], rtol=0, atol=1e-15)


def test_nonfinite_input_reported():
    require_gpu()
    m, x, v = ics.plummer(128, 2)
    x = x.copy()
    x[5, 1] = np.nan
    with pytest.raises(binding.NBodyError) as e:
        binding.NBody(m, x, v, eps=1e-3)
    assert e.value.code == binding.ENONFINITE


def test_mixed_block_steps_conserve_energy():
    # mixed path over block steps (Salpeter masses): single-evaluation parity
    # at the final state, and energy drift of the same order as FP64
    require_gpu()
    n = 4096
    m, x, v = ics.plummer(n, 3, masses=ics.salpeter_masses(n, 3))
    kw = dict(eps=1e-3, eta=0.02, level_min=4, level_max=20)
    res = {}
    for prec in (binding.FP64, binding.MIXED):
        g = binding.NBody(m, x, v, precision=prec, **kw)
        e0 = g.energy()[0]
        g.step(1 / 16)
        e1 = g.energy()[0]
        res[prec] = abs(e1[2] - e0[2]) / abs(e0[2])
        s = _state_np(g)
        a, j = (to_np(t) for t in g.forces(s["x"], s["v"], m))
        a_ref, j_ref = oracle.forces(s["x"], s["v"], m, 1e-3)
        check_parity(a, j, a_ref, j_ref, prec == binding.MIXED, "final state")
    assert res[binding.FP64] < 1e-4
    assert res[binding.MIXED] < 10 * res[binding.FP64] + 1e-7


def test_small_step_routing_tuning():
    # small_log2: 0 keeps the value, -1 turns the FP64 routing of small mixed
    # steps off, 1..62 set it; anything else is rejected on the host
    require_gpu()
    m, x, v = ics.plummer(512, 4)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.MIXED, level_min=5, level_max=20)
    assert g.get_tuning()["small_log2"] == 27
    g.set_tuning({"small_log2": 0})
    assert g.get_tuning()["small_log2"] == 27
    g.set_tuning({"small_log2": -1})
    assert g.get_tuning()["small_log2"] == -1
    st0 = g.stats()
    g.step(1 / 32)
    st1 = g.stats()
    assert st1["small_step_interactions"] == st0["small_step_interactions"]
    assert st1["interactions"] > st0["interactions"]
    g.set_tuning({"small_log2": 62})
    st2 = g.stats()
    g.step(1 / 16)
    st3 = g.stats()
    # every step of 512 particles is small: all of it on the FP64 kernel
    assert (st3["small_step_interactions"] - st2["small_step_interactions"]
            == st3["interactions"] - st2["interactions"] > 0)
    for bad in (63, -2, 200):
        with pytest.raises(binding.NBodyError) as e:
            g.set_tuning({"small_log2": bad})
        assert e.value.code == binding.EINVAL
    assert g.get_tuning()["small_log2"] == 62
