"""The acceleration-only force path (nbody_accel) and the paper's symplectic
drivers (nbody_step_symplectic: kick-drift-kick leapfrog and the
seven-stage sixth-order composition, Sect. 4) against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import FP64_TOL, MIXED_TOL, rel_err, require_gpu, to_np, is_mixed

pytestmark = pytest.mark.gpu

PRECS = [binding.FP64, binding.MIXED, binding.MIXED_DS]
SCHEMES = [binding.LEAPFROG, binding.SYMPLECTIC6]


def _tol(prec):
    return MIXED_TOL if is_mixed(prec) else FP64_TOL


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", [1, 2, 65, 257, 1000, 4097])
def test_accel_vs_oracle(n, prec):
    require_gpu()
    m, x, v = ics.plummer(n, 200 + n)
    m = ics.salpeter_masses(n, 300 + n) if n > 1 else m
    g = binding.NBody(m, x, v, eps=1e-3, precision=prec)
    acc = to_np(g.accel(x, m))
    g.sync()
    if n == 1:
        assert np.all(acc == 0)
        return
    a_ref, _ = oracle.forces(x, v, m, 1e-3)
    assert rel_err(acc, a_ref).max() <= _tol(prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("variant", [binding.VARIANT_K1, binding.VARIANT_K2,
                                     binding.VARIANT_S1, binding.VARIANT_S2])
def test_accel_equals_forces_acceleration_bitwise(prec, variant):
    # the acceleration-only pair term performs the same operations as the
    # acceleration part of the full one, on the same tiles and splits.  The
    # mixed full evaluation also takes its near pairs (chosen by their jerk
    # scale, which the acceleration-only path cannot see) in FP64: with near
    # pairs off the two agree bitwise, with them on both meet the oracle.
    require_gpu()
    n = 3000
    m, x, v = ics.plummer(n, 71)
    g = binding.NBody(m, x, v, eps=1e-4, precision=prec)
    g.set_tuning({"variant": variant})
    rng = np.random.default_rng(72)
    a_ref, _ = oracle.forces(x, v, m, 1e-4)
    for idx in (None, rng.integers(0, n, 500).astype(np.int32)):
        ref = a_ref if idx is None else a_ref[idx]
        if is_mixed(prec):
            a_near, _ = g.forces(x, v, m, i_active=idx)
            g.sync()
            assert rel_err(to_np(a_near), ref).max() <= _tol(prec)
            g.set_tuning({"near_jerk": -1.0})
        a_full, _ = g.forces(x, v, m, i_active=idx)
        a_only = g.accel(x, m, i_active=idx)
        g.sync()
        assert np.array_equal(to_np(a_full), to_np(a_only))
        assert rel_err(to_np(a_only), ref).max() <= _tol(prec)
        if is_mixed(prec):
            g.set_tuning({"near_jerk": 0.0625})


@pytest.mark.parametrize("prec", PRECS)
def test_accel_ensemble_and_zero_softening(prec):
    require_gpu()
    m, x, v, off = ics.ensemble(3, sizes=[300, 64, 700], seed=920)
    g = binding.NBody(m, x, v, eps=[1e-3, 0.0, 1e-4], precision=prec, cluster_offsets=off)
    acc = to_np(g.accel(x, m))
    g.sync()
    for c, eps in enumerate([1e-3, 0.0, 1e-4]):
        sl = slice(off[c], off[c + 1])
        a_ref, _ = oracle.forces(x[sl], v[sl], m[sl], eps)
        assert rel_err(acc[sl], a_ref).max() <= _tol(prec), c


def _positions_close(got, ref, tol):
    return np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_symplectic_fp64_matches_oracle(scheme):
    # Plummer N = 1024, eps = 1e-3, h = 1/256, 16 steps to t = 1/16
    require_gpu()
    n, h, steps = 1024, 1 / 256, 16
    m, x, v = ics.plummer(n, 1)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, level_min=4, level_max=20)
    ni = g.step_symplectic(scheme, h, steps)
    stages = 1 if scheme == binding.LEAPFROG else 7
    assert ni == (1 + steps * stages) * n * n
    s = {k: to_np(t) for k, t in g.get_state().items()}
    xr, vr = oracle.symplectic(x, v, m, 1e-3, h, steps, scheme)
    assert _positions_close(s["x"], xr, 1e-12)
    assert _positions_close(s["v"], vr, 1e-11)
    assert np.all(s["tick"] == (1 << 20) // 16)
    # the Hermite state is re-evaluated at the new positions
    a_ref, j_ref = oracle.forces(s["x"], s["v"], m, 1e-3)
    assert rel_err(s["a"], a_ref).max() <= FP64_TOL
    assert rel_err(s["j"], j_ref).max() <= FP64_TOL


@pytest.mark.parametrize("scheme", SCHEMES)
def test_symplectic_mixed_close_to_oracle(scheme):
    require_gpu()
    n, h, steps = 2048, 1 / 256, 16
    m, x, v = ics.plummer(n, 2)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.MIXED, level_min=4, level_max=20)
    g.step_symplectic(scheme, h, steps)
    s = {k: to_np(t) for k, t in g.get_state().items()}
    xr, vr = oracle.symplectic(x, v, m, 1e-3, h, steps, scheme)
    # acceleration errors of at most 1e-6 |a| move v by at most that times
    # the elapsed time t and x by at most half of it times t^2 (factor 2 of
    # headroom for the change of |a| along the orbit)
    t = h * steps
    amax = np.linalg.norm(oracle.forces(x, v, m, 1e-3)[0], axis=1).max()
    assert np.abs(s["v"] - vr).max() <= 2 * MIXED_TOL * amax * t
    assert np.abs(s["x"] - xr).max() <= MIXED_TOL * amax * t * t


def test_symplectic_time_reversible_on_gpu():
    require_gpu()
    n, h, steps = 512, 1 / 256, 16
    m, x, v = ics.plummer(n, 3)
    g = binding.NBody(m, x, v, eps=1e-2, precision=binding.FP64, level_min=4, level_max=20)
    g.step_symplectic(binding.SYMPLECTIC6, h, steps)
    s = g.get_state()
    s["v"] = -s["v"]
    g.set_state(s)
    g.step_symplectic(binding.SYMPLECTIC6, h, steps)
    s2 = {k: to_np(t) for k, t in g.get_state().items()}
    assert _positions_close(s2["x"], x, 1e-12)
    assert _positions_close(-s2["v"], v, 1e-11)


def test_symplectic_ensemble_per_cluster():
    require_gpu()
    m, x, v, off = ics.ensemble(3, sizes=[300, 64, 513], seed=930)
    eps = [1e-3, 2e-3, 1e-4]
    g = binding.NBody(m, x, v, eps=eps, precision=binding.FP64, cluster_offsets=off,
                      level_min=4, level_max=20)
    g.step_symplectic(binding.LEAPFROG, 1 / 128, 8)
    s = {k: to_np(t) for k, t in g.get_state().items()}
    for c in range(3):
        sl = slice(off[c], off[c + 1])
        xr, vr = oracle.symplectic(x[sl], v[sl], m[sl], eps[c], 1 / 128, 8, binding.LEAPFROG)
        assert _positions_close(s["x"][sl], xr, 1e-12), c
        assert _positions_close(s["v"][sl], vr, 1e-11), c


def test_symplectic_then_block_steps_and_energy():
    # leapfrog keeps the energy error bounded; block steps can follow
    require_gpu()
    n = 1024
    m, x, v = ics.plummer(n, 4)
    g = binding.NBody(m, x, v, eps=1e-2, precision=binding.MIXED, level_min=3, level_max=20)
    e0 = g.energy()[0, 2]
    g.step_symplectic(binding.LEAPFROG, 1 / 512, 64)
    e1 = g.energy()[0, 2]
    assert abs(e1 - e0) <= 1e-4 * abs(e0)
    g.step(0.25)
    e2 = g.energy()[0, 2]
    assert abs(e2 - e0) <= 1e-4 * abs(e0)
    assert np.all(to_np(g.get_state()["tick"]) == (1 << 20) // 4)


def test_symplectic_rejects_bad_arguments():
    require_gpu()
    m, x, v = ics.plummer(64, 5)
    g = binding.NBody(m, x, v, eps=1e-2, precision=binding.FP64, level_min=4, level_max=6)
    for args in ((7, 1 / 64, 4), (binding.LEAPFROG, 1e-3, 4), (binding.LEAPFROG, 1 / 64, 3),
                 (binding.LEAPFROG, -1 / 64, 4), (binding.LEAPFROG, 1 / 64, -1)):
        with pytest.raises(binding.NBodyError) as e:
            g.step_symplectic(*args)
        assert e.value.code == binding.EINVAL, args
    # a particle in the middle of its block step
    s = g.get_state()
    level = np.full(64, 5, np.int8)
    level[0] = 4
    tick = np.full(64, 1 << 15, np.int64)
    tick[0] = 0
    s["level"], s["tick"] = level, tick
    g.set_state(s)
    with pytest.raises(binding.NBodyError) as e:
        g.step_symplectic(binding.LEAPFROG, 1 / 64, 4)
    assert e.value.code == binding.EINVAL


@pytest.mark.parametrize("prec", PRECS)
def test_symplectic_graph_replay_equals_eager_bitwise(prec):
    # steps after the first replay one captured graph; with profiling on
    # every launch is eager: both must give the same bits
    require_gpu()
    m, x, v = ics.plummer(700, 6)
    out = []
    for profile in (False, True):
        g = binding.NBody(m, x, v, eps=1e-3, precision=prec, level_min=4, level_max=20)
        g.profile(profile)
        g.step_symplectic(binding.SYMPLECTIC6, 1 / 256, 16)
        out.append({k: to_np(t) for k, t in g.get_state().items()})
        g.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


@pytest.mark.parametrize("prec", PRECS)
def test_acc_variant_is_independent_of_variant(prec):
    # the acceleration-only evaluations take their own kernel variant; each
    # combination stays within the oracle's tolerance, block steps keep
    # theirs, and -1 returns the field to "the same as variant"
    require_gpu()
    n = 3000
    m, x, v = ics.plummer(n, 73)
    a_ref, j_ref = oracle.forces(x, v, m, 1e-4)
    g = binding.NBody(m, x, v, eps=1e-4, precision=prec)
    for var, acc_var in ((binding.VARIANT_K1, binding.VARIANT_K2),
                         (binding.VARIANT_K2, binding.VARIANT_S1),
                         (binding.VARIANT_S2, binding.VARIANT_K1)):
        g.set_tuning({"variant": var, "acc_variant": acc_var})
        t = g.get_tuning()
        assert t["variant"] == var and t["acc_variant"] == acc_var
        acc = to_np(g.accel(x, m))
        a_full, j_full = g.forces(x, v, m)
        g.sync()
        assert rel_err(acc, a_ref).max() <= _tol(prec)
        assert rel_err(to_np(a_full), a_ref).max() <= _tol(prec)
    g.set_tuning({"acc_variant": -1})
    assert g.get_tuning()["acc_variant"] == 0
    with pytest.raises(binding.NBodyError) as e:
        g.set_tuning({"acc_variant": 7})
    assert e.value.code == binding.EINVAL


def test_symplectic_with_other_acc_variant_matches_oracle():
    require_gpu()
    n, h, steps = 1024, 1 / 256, 16
    m, x, v = ics.plummer(n, 1)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, level_min=4, level_max=20)
    g.set_tuning({"variant": binding.VARIANT_K1, "acc_variant": binding.VARIANT_S2})
    g.step_symplectic(binding.SYMPLECTIC6, h, steps)
    s = {k: to_np(t) for k, t in g.get_state().items()}
    xr, vr = oracle.symplectic(x, v, m, 1e-3, h, steps, binding.SYMPLECTIC6)
    assert _positions_close(s["x"], xr, 1e-12)
    assert _positions_close(s["v"], vr, 1e-11)
    a_ref, j_ref = oracle.forces(s["x"], s["v"], m, 1e-3)
    assert rel_err(s["a"], a_ref).max() <= FP64_TOL
    assert rel_err(s["j"], j_ref).max() <= FP64_TOL
