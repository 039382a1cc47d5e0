"""Parity of nbody_forces (HIP, through the C ABI) against the CPU oracle:
eq. (1) with Plummer softening plus jerk, FP64 path within 1e-12 and mixed
path within 1e-6 relative per particle, over ragged sizes, subsets with
repeats, zero softening, ensembles and the error paths."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import (FP64_TOL, MIXED_TOL, check_parity, is_mixed,
                            rel_err, require_gpu, to_np)

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 255, 256, 257, 513, 1000, 1024, 4097]


def _ctx(m, x, v, eps, prec, **kw):
    return binding.NBody(m, x, v, eps=eps, precision=prec, **kw)


PRECS = [binding.FP64, binding.MIXED, binding.MIXED_DS]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", SIZES)
def test_all_particles_vs_oracle(n, prec):
    require_gpu()
    print(f"forces n={n} prec={prec}", flush=True)
    m, x, v = ics.plummer(n, 100 + n)
    eps = 1e-3
    g = _ctx(m, x, v, eps, prec)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, eps)
    if n == 1:
        assert np.all(to_np(acc) == 0) and np.all(to_np(jerk) == 0)
        return
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec), f"n={n}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("na", [1, 2, 5, 17, 100, 700, 3000])
def test_subsets_with_repeats(na, prec):
    require_gpu()
    n = 2500
    m, x, v = ics.plummer(n, 7)
    m = ics.salpeter_masses(n, 8)          # uneven masses
    rng = np.random.default_rng(na)
    idx = rng.integers(0, n, na).astype(np.int32)
    idx[: min(3, na)] = idx[0]             # repeats
    g = _ctx(m, x, v, 1e-4, prec)
    acc, jerk = g.forces(x, v, m, i_active=idx)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 1e-4, idx=idx.astype(np.int64))
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec), f"na={na}")


@pytest.mark.parametrize("prec", PRECS)
def test_j_set_larger_than_context(prec):
    # one cluster: n_j is free, independent of the context's n
    require_gpu()
    m0, x0, v0 = ics.plummer(64, 1)
    g = _ctx(m0, x0, v0, 1e-3, prec)
    m, x, v = ics.plummer(20000, 2)
    idx = np.arange(0, 20000, 37, dtype=np.int32)
    acc, jerk = g.forces(x, v, m, i_active=idx)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 1e-3, idx=idx.astype(np.int64))
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec))


@pytest.mark.parametrize("prec", PRECS)
def test_j_set_of_2_23(prec):
    # one cluster of 2^23 j, eight times the largest benchmark system: 64-bit
    # j offsets and long split ranges; sampled i, the last index among them
    require_gpu()
    n = 1 << 23
    m0, x0, v0 = ics.plummer(64, 1)
    g = _ctx(m0, x0, v0, 1e-4, prec)
    m, x, v = ics.plummer(n, 23)
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(n - 1, 255, replace=False))
    idx = np.append(idx, n - 1).astype(np.int32)
    print(f"n_j 2^23 prec={prec}", flush=True)
    acc, jerk = g.forces(x, v, m, i_active=idx)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 1e-4, idx=idx.astype(np.int64))
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec), "n_j 2^23")


@pytest.mark.parametrize("prec", PRECS)
def test_zero_softening(prec):
    require_gpu()
    rng = np.random.default_rng(3)
    x = rng.normal(size=(300, 3))
    v = rng.normal(size=(300, 3))
    m = rng.uniform(0.1, 1.0, 300)
    g = _ctx(m, x, v, 0.0, prec)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 0.0)
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec))


def test_zero_softening_coincident_is_edomain():
    require_gpu()
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0]])
    v = np.zeros((3, 3))
    m = np.ones(3)
    g = _ctx(np.ones(2), x[:2], v[:2], 0.0, binding.FP64)
    g.forces(x, v, m)
    with pytest.raises(binding.NBodyError) as e:
        g.sync()
    assert e.value.code == binding.EDOMAIN
    g.sync()      # error is cleared once reported


def test_index_out_of_range_is_eindex():
    require_gpu()
    m, x, v = ics.plummer(100, 4)
    g = _ctx(m, x, v, 1e-3, binding.FP64)
    acc, jerk = g.forces(x, v, m, i_active=np.array([0, 5, 100, -1, 7], np.int32))
    with pytest.raises(binding.NBodyError) as e:
        g.sync()
    assert e.value.code == binding.EINDEX
    a = to_np(acc)
    assert np.all(a[2] == 0) and np.all(a[3] == 0)
    a_ref, _ = oracle.forces(x, v, m, 1e-3, idx=np.array([0, 5, 7]))
    assert rel_err(a[[0, 1, 4]], a_ref).max() <= FP64_TOL


@pytest.mark.parametrize("prec", PRECS)
def test_ensemble_forces_per_cluster(prec):
    tol = MIXED_TOL if is_mixed(prec) else FP64_TOL
    require_gpu()
    m, x, v, off = ics.ensemble(5, sizes=[257, 64, 1000, 3, 511], seed=900)
    eps = [1e-3, 2e-3, 1e-4, 1e-3, 5e-4]
    g = _ctx(m, x, v, eps, prec, cluster_offsets=off)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a, j = to_np(acc), to_np(jerk)
    for c in range(5):
        sl = slice(off[c], off[c + 1])
        a_ref, j_ref = oracle.forces(x[sl], v[sl], m[sl], eps[c])
        check_parity(a[sl], j[sl], a_ref, j_ref, is_mixed(prec), f"cluster {c}")
    # grouped subset with repeats, skipping cluster 1 entirely
    idx = np.array([0, 0, 5, 400, 400, 1321, 1322, 1400], np.int32)
    acc, jerk = g.forces(x, v, m, i_active=idx)
    g.sync()
    cl = np.searchsorted(off, idx, side="right") - 1
    for k, i in enumerate(idx):
        c = cl[k]
        sl = slice(off[c], off[c + 1])
        a_ref, _ = oracle.forces(x[sl], v[sl], m[sl], eps[c], idx=[i - off[c]])
        assert rel_err(to_np(acc)[k:k + 1], a_ref).max() <= tol
    # not grouped by cluster
    g.forces(x, v, m, i_active=np.array([400, 0], np.int32))
    with pytest.raises(binding.NBodyError) as e:
        g.sync()
    assert e.value.code == binding.EINDEX


@pytest.mark.parametrize("prec,tol,jtol", [(binding.FP64, 1e-14, 1e-13),
                                           (binding.MIXED, MIXED_TOL, MIXED_TOL),
                                           (binding.MIXED_DS, MIXED_TOL, MIXED_TOL)])
def test_split_and_tile_shape_invariance(prec, tol, jtol):
    # every launch shape sums the same terms in another order (and, on the
    # mixed path, may re-evaluate a slightly different set in FP64)
    require_gpu()
    m, x, v = ics.plummer(6000, 5)
    g = _ctx(m, x, v, 1e-3, prec)
    idx = np.arange(0, 6000, 3, dtype=np.int32)[:150]
    base_a, base_j = (to_np(t) for t in g.forces(x, v, m, i_active=idx))
    for variant in (binding.VARIANT_K1, binding.VARIANT_K2, binding.VARIANT_S1,
                    binding.VARIANT_S2):
        for slots, target in ((1, 1), (4, 64), (64, 4096), (256, 1)):
            g.set_tuning({"variant": variant, "i_slots": [slots] * 25,
                          "target_items": [target] * 25, "min_split_j": 64})
            a, j = (to_np(t) for t in g.forces(x, v, m, i_active=idx))
            assert rel_err(a, base_a).max() <= tol, (variant, slots, target)
            assert rel_err(j, base_j).max() <= jtol, (variant, slots, target)


@pytest.mark.parametrize("prec", PRECS)
def test_full_evaluation_at_the_partial_row_bound(prec):
    # every particle active with the largest split target: the plan cuts j
    # into 32 chunks of 256 (32 partial rows per particle, the workspace
    # bound) and hands the items out split-major; every variant against the
    # oracle, and per K the broadcast kernel = the workgroup kernel bitwise
    require_gpu()
    n = 8192
    m, x, v = ics.plummer(n, 21)
    a_ref, j_ref = oracle.forces(x, v, m, 1e-3)
    g = _ctx(m, x, v, 1e-3, prec)
    got = {}
    for variant in (binding.VARIANT_K1, binding.VARIANT_K2, binding.VARIANT_S1,
                    binding.VARIANT_S2):
        print(f"partial-row bound n={n} prec={prec} variant={variant}", flush=True)
        g.set_tuning({"variant": variant, "i_slots": [256] * 25,
                      "target_items": [1 << 20] * 25, "min_split_j": 64})
        a, j = (to_np(t) for t in g.forces(x, v, m))
        check_parity(a, j, a_ref, j_ref, is_mixed(prec), f"variant {variant}")
        got[variant] = (a, j)
    for lds, sb in ((binding.VARIANT_K1, binding.VARIANT_S1),
                    (binding.VARIANT_K2, binding.VARIANT_S2)):
        assert np.array_equal(got[lds][0], got[sb][0])
        assert np.array_equal(got[lds][1], got[sb][1])
    # an ensemble at the same bound: the clusters' rows add up to at most
    # 32 per particle of the context
    m, x, v, off = ics.ensemble(4, sizes=[4096, 300, 2048, 1537], seed=901)
    eps = [1e-3, 2e-3, 1e-3, 5e-4]
    ge = _ctx(m, x, v, eps, prec, cluster_offsets=off)
    ge.set_tuning({"variant": binding.VARIANT_S1, "i_slots": [256] * 25,
                   "target_items": [1 << 20] * 25, "min_split_j": 64})
    acc, jerk = ge.forces(x, v, m)
    a, j = to_np(acc), to_np(jerk)
    for c in range(4):
        sl = slice(off[c], off[c + 1])
        a_ref, j_ref = oracle.forces(x[sl], v[sl], m[sl], eps[c])
        check_parity(a[sl], j[sl], a_ref, j_ref, is_mixed(prec), f"cluster {c}")


@pytest.mark.parametrize("prec", PRECS)
def test_bitwise_deterministic(prec):
    require_gpu()
    m, x, v = ics.plummer(3000, 6)
    g = _ctx(m, x, v, 1e-3, prec)
    idx = np.arange(0, 3000, 7, dtype=np.int32)
    r1 = [to_np(t) for t in g.forces(x, v, m, i_active=idx)]
    r2 = [to_np(t) for t in g.forces(x, v, m, i_active=idx)]
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


def test_mixed_within_fp64_path():
    # both GPU paths at identical inputs; the mixed one within 1e-6 of FP64
    require_gpu()
    m, x, v = ics.plummer(8192, 9)
    m = ics.salpeter_masses(8192, 10)
    g64 = _ctx(m, x, v, 1e-4, binding.FP64)
    gm = _ctx(m, x, v, 1e-4, binding.MIXED)
    a64, j64 = (to_np(t) for t in g64.forces(x, v, m))
    am, jm = (to_np(t) for t in gm.forces(x, v, m))
    check_parity(am, jm, a64, j64, True, "mixed vs fp64 gpu")


@pytest.mark.parametrize("kind", ["plummer", "king"])
def test_mixed_refines_few_particles(kind):
    # the FP64 re-evaluation is for the few particles dominated by one
    # neighbour; the self slot must not count as a neighbour
    require_gpu()
    n = 16384
    m, x, v = ics.plummer(n, 12) if kind == "plummer" else ics.king(n, 7.0, 13)
    eps = 1e-3 if kind == "plummer" else 1e-4
    g = _ctx(m, x, v, eps, binding.MIXED)
    r0 = g.stats()["refined"]
    acc, jerk = g.forces(x, v, m)
    refined = g.stats()["refined"] - r0
    print(f"  {kind}: {refined} of {n} re-evaluated in FP64", flush=True)
    assert refined < 0.05 * n
    a_ref, j_ref = oracle.forces(x, v, m, eps)
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, True, kind)


def test_mixed_refines_dominated_particles_in_fp64():
    # a tight pair inside a cluster: the members' accelerations are dominated
    # by each other, so the mixed path re-evaluates them with the FP64 kernel
    require_gpu()
    m, x, v = ics.plummer(2048, 31)
    x = x.copy()
    x[1] = x[0] + np.array([3e-4, -2e-4, 1e-4])
    g = _ctx(m, x, v, 1e-5, binding.MIXED)
    # the pair term is about the whole acceleration: flag at half of it
    g.set_tuning({"refine_ratio": 0.5})
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 1e-5)
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, True, "with tight pair")
    assert rel_err(to_np(acc)[:2], a_ref[:2]).max() <= 1e-12
    assert rel_err(to_np(jerk)[:2], j_ref[:2]).max() <= 1e-12
    # without the re-evaluation the pure FP32 path is still within 1e-6 on
    # the median particle
    g.set_tuning({"refine_ratio": -1.0})
    acc2, jerk2 = g.forces(x, v, m)
    g.sync()
    assert np.median(rel_err(to_np(acc2), a_ref)) <= 1e-7
    assert rel_err(to_np(acc2)[:2], a_ref[:2]).max() > 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_more_clusters_than_plan_threads(prec):
    # 4096 clusters (the maximum): the plan's threads each own four clusters
    require_gpu()
    rng = np.random.default_rng(77)
    nc = 4096                      # the largest cluster count a context takes
    sizes = rng.integers(2, 12, nc).tolist()
    m, x, v, off = ics.ensemble(nc, sizes=sizes, seed=940)
    eps = rng.uniform(1e-3, 1e-2, nc)
    g = _ctx(m, x, v, list(eps), prec, cluster_offsets=off)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a, j = to_np(acc), to_np(jerk)
    worst_a = worst_j = 0.0
    for c in range(nc):
        sl = slice(off[c], off[c + 1])
        a_ref, j_ref = oracle.forces(x[sl], v[sl], m[sl], eps[c])
        worst_a = max(worst_a, rel_err(a[sl], a_ref).max())
        worst_j = max(worst_j, rel_err(j[sl], j_ref).max())
    tol = MIXED_TOL if is_mixed(prec) else FP64_TOL
    jtol = MIXED_TOL if is_mixed(prec) else FP64_TOL
    assert worst_a <= tol and worst_j <= jtol, (worst_a, worst_j)
    # block steps run the plan every step
    e0 = g.energy()[:, 2]
    g.step(0.125)
    e1 = g.energy()[:, 2]
    assert np.all(np.isfinite(e1))
    assert np.median(np.abs(e1 - e0) / np.abs(e0)) < 1e-5


def test_empty_active_set_is_a_no_op():
    require_gpu()
    m, x, v = ics.plummer(64, 41)
    g = _ctx(m, x, v, 1e-3, binding.MIXED)
    acc, jerk = g.forces(x, v, m, i_active=np.zeros(0, np.int32))
    g.sync()
    assert acc.shape == (0, 3) and jerk.shape == (0, 3)


@pytest.mark.parametrize("prec", PRECS)
def test_massless_tracers(prec):
    # zero-mass particles feel the field and exert none
    require_gpu()
    m, x, v = ics.plummer(1500, 42)
    m = m.copy()
    m[::3] = 0.0
    g = _ctx(m, x, v, 1e-3, prec)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    a_ref, j_ref = oracle.forces(x, v, m, 1e-3)
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, is_mixed(prec), "tracers")
    # the massive particles' forces do not depend on the tracers at all
    heavy = np.nonzero(m > 0)[0]
    a_h, j_h = oracle.forces(x[heavy], v[heavy], m[heavy], 1e-3)
    check_parity(to_np(acc)[heavy], to_np(jerk)[heavy], a_h, j_h, is_mixed(prec),
                 "tracers removed")
