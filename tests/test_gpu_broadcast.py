"""The broadcast force kernel (j records in scalar registers) against the
workgroup kernel that stages j through LDS.  Both evaluate eq. (1) plus jerk
with the same operations in the same order per (i, j-chunk), so with the same
i-particles per lane (K) their results are bitwise identical; against the
oracle they meet the usual parity bar.  Covered: nbody_forces (caller's
arrays), the initial evaluation, block steps (records predicted on the
device), ensembles, zero softening, and the index check on caller input."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import check_parity, require_gpu, to_np, is_mixed

pytestmark = pytest.mark.gpu

PAIRS = [(binding.VARIANT_K1, binding.VARIANT_S1), (binding.VARIANT_K2, binding.VARIANT_S2)]
PRECS = [binding.FP64, binding.MIXED, binding.MIXED_DS]
WIDE = {"i_slots": [256] * 25}       # kWG i-slots in every bucket: broadcast-eligible


def _forces(g, x, v, m, idx=None):
    a, j = g.forces(x, v, m, i_active=idx)
    g.sync()
    return to_np(a), to_np(j)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("lds,sb", PAIRS)
def test_forces_bitwise_equal_to_lds_kernel(prec, lds, sb):
    require_gpu()
    n = 3000
    m, x, v = ics.plummer(n, 61)
    m = ics.salpeter_masses(n, 62)
    g = binding.NBody(m, x, v, eps=1e-4, precision=prec)
    rng = np.random.default_rng(63)
    for idx in (None, np.sort(rng.choice(n, 700, replace=False)).astype(np.int32),
                rng.integers(0, n, 400).astype(np.int32)):       # unsorted, repeats
        g.set_tuning({"variant": lds, **WIDE})
        a0, j0 = _forces(g, x, v, m, idx)
        g.set_tuning({"variant": sb, **WIDE})
        a1, j1 = _forces(g, x, v, m, idx)
        assert np.array_equal(a0, a1) and np.array_equal(j0, j1)
        sel = np.arange(n) if idx is None else idx.astype(np.int64)
        a_ref, j_ref = oracle.forces(x, v, m, 1e-4, idx=sel)
        check_parity(a1, j1, a_ref, j_ref, is_mixed(prec), f"variant {sb}")


@pytest.mark.parametrize("prec", PRECS)
def test_zero_softening_bitwise_and_edomain(prec):
    require_gpu()
    rng = np.random.default_rng(64)
    x, v = rng.normal(size=(700, 3)), rng.normal(size=(700, 3))
    m = rng.uniform(0.1, 1.0, 700)
    g = binding.NBody(m, x, v, eps=0.0, precision=prec)
    out = []
    for var in (binding.VARIANT_K1, binding.VARIANT_S1):
        g.set_tuning({"variant": var, **WIDE})
        out.append(_forces(g, x, v, m))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    a_ref, j_ref = oracle.forces(x, v, m, 0.0)
    check_parity(out[1][0], out[1][1], a_ref, j_ref, is_mixed(prec), "eps=0")
    # two distinct coincident particles
    x2 = x.copy()
    x2[5] = x2[9]
    g.forces(x2, v, m)
    with pytest.raises(binding.NBodyError) as e:
        g.sync()
    assert e.value.code == binding.EDOMAIN


def test_index_out_of_range_is_eindex():
    require_gpu()
    m, x, v = ics.plummer(64, 65)
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.MIXED)
    g.set_tuning({"variant": binding.VARIANT_S1, **WIDE})
    idx = np.array([0, 5, 64, -1, 7, 8, 9, 10], np.int32)   # 8 >= 64 / 16: records built
    acc, jerk = g.forces(x, v, m, i_active=idx)
    with pytest.raises(binding.NBodyError) as e:
        g.sync()
    assert e.value.code == binding.EINDEX
    a = to_np(acc)
    assert np.all(a[2] == 0) and np.all(a[3] == 0)
    good = [0, 1, 4, 5, 6, 7]
    a_ref, j_ref = oracle.forces(x, v, m, 1e-3, idx=idx[good].astype(np.int64))
    check_parity(a[good], to_np(jerk)[good], a_ref, j_ref, True, "valid entries")


@pytest.mark.parametrize("prec", PRECS)
def test_ensemble_bitwise_equal_to_lds_kernel(prec):
    require_gpu()
    m, x, v, off = ics.ensemble(4, sizes=[700, 300, 1200, 513], seed=910)
    eps = [1e-3, 2e-3, 1e-4, 5e-4]
    g = binding.NBody(m, x, v, eps=eps, precision=prec, cluster_offsets=off)
    out = []
    for var in (binding.VARIANT_K1, binding.VARIANT_S1):
        g.set_tuning({"variant": var, **WIDE})
        out.append(_forces(g, x, v, m))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    for c in range(4):
        sl = slice(off[c], off[c + 1])
        a_ref, j_ref = oracle.forces(x[sl], v[sl], m[sl], eps[c])
        check_parity(out[1][0][sl], out[1][1][sl], a_ref, j_ref, is_mixed(prec),
                     f"cluster {c}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("lds,sb", PAIRS)
def test_block_steps_bitwise_equal_to_lds_kernel(prec, lds, sb):
    # block steps mix large steps (records predicted on the device, broadcast
    # kernel) with small ones (prediction fused into the LDS tile fill)
    require_gpu()
    n = 4096
    m, x, v = ics.plummer(n, 66)
    kw = dict(eps=1e-3, precision=prec, eta=0.02, eta_start=0.01, level_min=4, level_max=20)
    states = []
    for var in (lds, sb):
        g = binding.NBody(m, x, v, tuning={"variant": var, **WIDE}, **kw)
        ns, ni = g.step(1 / 16)
        states.append((ns, ni, {k: to_np(t) for k, t in g.get_state().items()}))
        g.close()
    (ns0, ni0, s0), (ns1, ni1, s1) = states
    assert ns0 == ns1 and ni0 == ni1 and ns0 > 16
    for k in s0:
        assert np.array_equal(s0[k], s1[k]), k
