"""The external Galactic field (the Allen & Santillan model the paper adds to
the pairwise forces, Sect. 4) on the GPU against the CPU oracle: initial
acceleration, jerk and levels, Hermite block steps, the symplectic drivers
and the energy, for a star cluster on a Galactic orbit; a single star on a
circular orbit; ensembles; the field switched off."""
import math

import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import FP64_TOL, check_parity, rel_err, require_gpu, to_np

pytestmark = pytest.mark.gpu

MASS_MSUN, LENGTH_KPC = 1e5, 1e-3        # cluster units: 1e5 M_sun, 1 pc
R_SUN_KPC = 8.5


def _field():
    return binding.allen_santillan(length_unit_kpc=LENGTH_KPC, mass_unit_msun=MASS_MSUN)


def _cluster(n, seed, field, phase=0.0):
    """Plummer cluster (Henon units) on a circular orbit at the Sun's radius."""
    R = R_SUN_KPC / LENGTH_KPC
    acc, _, _ = oracle.field_eval(field, [R, 0.0, 0.0], [0.0, 0.0, 0.0])
    vc = math.sqrt(R * -acc[0])
    m, x, v = ics.plummer(n, seed)
    c, s = math.cos(phase), math.sin(phase)
    x = x + np.array([R * c, R * s, 0.0])
    v = v + np.array([-vc * s, vc * c, 0.0])
    return m, x, v


def _state(g):
    return {k: to_np(t) for k, t in g.get_state().items()}


@pytest.mark.parametrize("prec", [binding.FP64, binding.MIXED])
def test_initial_state_with_field_matches_oracle(prec):
    require_gpu()
    f = _field()
    m, x, v = _cluster(2000, 40, f)
    g = binding.NBody(m, x, v, eps=1e-3, precision=prec, eta=0.01, eta_start=0.01,
                      level_min=3, level_max=20, field=f)
    s = _state(g)
    ref = oracle.System(m, x, v, 1e-3, eta=0.01, eta_start=0.01, level_min=3, level_max=20,
                        field=f)
    check_parity(s["a"], s["j"], ref.a, ref.j, prec == binding.MIXED, "init with field")
    if prec == binding.FP64:
        assert np.array_equal(s["level"].astype(np.int64), ref.level.astype(np.int64))
    # the field is in there: without it the stored values differ
    free = binding.NBody(m, x, v, eps=1e-3, precision=prec, level_min=3, level_max=20)
    assert rel_err(_state(free)["a"], ref.a).max() > 1e-3


@pytest.mark.parametrize("n,t_end,lmin", [(300, 0.125, 3), (1200, 0.0625, 4)])
def test_block_steps_with_field_match_oracle(n, t_end, lmin):
    require_gpu()
    print(f"field block steps n={n}", flush=True)
    f = _field()
    m, x, v = _cluster(n, 41 + n, f)
    kw = dict(eta=0.02, eta_start=0.01, level_min=lmin, level_max=20)
    g = binding.NBody(m, x, v, eps=1e-2, precision=binding.FP64, field=f, **kw)
    ns, _ = g.step(t_end)
    s = _state(g)
    ref = oracle.System(m, x, v, 1e-2, field=f, **kw)
    ref.run(t_end)
    assert ns == ref.stats.n_block_steps
    assert np.array_equal(s["level"].astype(np.int64), ref.level.astype(np.int64))
    assert np.all(s["tick"] == ref.tick)
    # positions about 8500 from the Galactic centre: compare the offsets
    c = np.array([R_SUN_KPC / LENGTH_KPC, 0.0, 0.0])
    assert np.abs((s["x"] - c) - (ref.x - c)).max() <= 1e-9
    assert np.abs(s["v"] - ref.v).max() <= 1e-8
    assert rel_err(s["a"], ref.a).max() <= 1e-9
    assert len(np.unique(s["level"])) > 1


def test_mixed_block_steps_with_field_conserve_energy():
    require_gpu()
    f = _field()
    m, x, v = _cluster(4096, 43, f)
    e = {}
    for prec in (binding.FP64, binding.MIXED):
        g = binding.NBody(m, x, v, eps=1e-3, precision=prec, eta=0.02, level_min=3,
                          level_max=20, field=f)
        e0 = g.energy()[0]
        g.step(1 / 8)
        e1 = g.energy()[0]
        e[prec] = abs(e1[2] - e0[2]) / abs(e0[1])      # relative to the cluster's |W|
        assert abs(e1[5] - e0[5]) <= 1e-9 * abs(e0[5])   # L_z: the field is axisymmetric
    assert e[binding.FP64] < 1e-4
    assert e[binding.MIXED] < 10 * e[binding.FP64] + 1e-7


@pytest.mark.parametrize("scheme", [binding.LEAPFROG, binding.SYMPLECTIC6])
def test_symplectic_with_field_matches_oracle(scheme):
    require_gpu()
    f = _field()
    m, x, v = _cluster(512, 44, f)
    n, h, steps = 512, 1 / 256, 16
    g = binding.NBody(m, x, v, eps=1e-3, precision=binding.FP64, level_min=4, level_max=20,
                      field=f)
    g.step_symplectic(scheme, h, steps)
    s = _state(g)
    xr, vr = oracle.symplectic(x, v, m, 1e-3, h, steps, scheme, field=f)
    c = np.array([R_SUN_KPC / LENGTH_KPC, 0.0, 0.0])
    assert np.abs((s["x"] - c) - (xr - c)).max() <= 1e-11
    assert np.abs(s["v"] - vr).max() <= 1e-10
    # the closing Hermite evaluation includes the field
    ref = oracle.System(m, s["x"], s["v"], 1e-3, level_min=4, level_max=20, field=f)
    assert rel_err(s["a"], ref.a).max() <= FP64_TOL
    assert rel_err(s["j"], ref.j).max() <= FP64_TOL
    assert n == m.shape[0]


def test_energy_with_field_matches_oracle():
    require_gpu()
    f = _field()
    m, x, v = _cluster(3000, 45, f)
    for prec in (binding.FP64, binding.MIXED):
        g = binding.NBody(m, x, v, eps=1e-3, precision=prec, field=f)
        e = g.energy()[0]
        r = oracle.energy(x, v, m, 1e-3, field=f)
        assert abs(e[0] - r["K"]) <= 1e-14 * abs(r["K"])
        assert abs(e[1] - r["W"]) <= 1e-13 * abs(r["W"])
        assert abs(e[2] - r["E"]) <= 1e-13 * abs(r["E"])
        assert abs(e[2] - e[0] - e[1]) > 1.0            # the field's potential energy


def test_single_star_circular_orbit():
    # one star in the model's own units (kpc, 2.32e7 M_sun): shared steps of
    # 2^-7 over about one orbit, against the oracle and the exact circle
    require_gpu()
    f = binding.allen_santillan()
    R = R_SUN_KPC
    acc, _, _ = oracle.field_eval(f, [R, 0.0, 0.0], [0.0, 0.0, 0.0])
    vc = math.sqrt(R * -acc[0])
    m, x, v = np.array([1e-12]), np.array([[R, 0.0, 0.0]]), np.array([[0.0, vc, 0.0]])
    kw = dict(dt_shared=2.0 ** -7, level_min=1, level_max=20)
    g = binding.NBody(m, x, v, eps=0.0, precision=binding.FP64, field=f, **kw)
    g.step(2.5)
    s = _state(g)
    ref = oracle.System(m, x, v, 0.0, field=f, **kw)
    ref.run(2.5)
    assert np.abs(s["x"] - ref.x).max() <= 1e-12 * R
    om = vc / R
    exact = R * np.array([math.cos(2.5 * om), math.sin(2.5 * om), 0.0])
    assert np.linalg.norm(s["x"][0] - exact) <= 1e-6 * R


@pytest.mark.parametrize("prec", [binding.FP64, binding.MIXED])
def test_ensemble_with_field_equals_solo_bitwise(prec):
    require_gpu()
    f = _field()
    parts = [_cluster(nc, 46 + k, f, phase=k * 2.0) for k, nc in enumerate((300, 64, 513))]
    m = np.concatenate([p[0] for p in parts])
    x = np.concatenate([p[1] for p in parts])
    v = np.concatenate([p[2] for p in parts])
    off = np.cumsum([0] + [p[0].shape[0] for p in parts])
    kw = dict(precision=prec, eta=0.02, level_min=4, level_max=20, field=f)
    g = binding.NBody(m, x, v, eps=[1e-3] * 3, cluster_offsets=off, **kw)
    g.step(1 / 16)
    s = _state(g)
    for c, (mc, xc, vc) in enumerate(parts):
        solo = binding.NBody(mc, xc, vc, eps=1e-3, **kw)
        solo.step(1 / 16)
        ss = _state(solo)
        sl = slice(off[c], off[c + 1])
        for k in ("x", "v", "a", "j", "tick", "level"):
            assert np.array_equal(s[k][sl], ss[k]), (c, k)


def test_zero_mass_field_equals_no_field_bitwise():
    require_gpu()
    m, x, v = ics.plummer(700, 47)
    kw = dict(eps=1e-2, precision=binding.MIXED, eta=0.02, level_min=4, level_max=20)
    a = binding.NBody(m, x, v, **kw)
    b = binding.NBody(m, x, v, field={"bulge_m": 0.0, "disk_m": 0.0, "halo_m": 0.0}, **kw)
    a.step(1 / 16)
    b.step(1 / 16)
    sa, sb = _state(a), _state(b)
    for k in ("x", "v", "a", "j", "tick", "level"):
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.energy(), b.energy())
