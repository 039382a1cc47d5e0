"""Seeded input generators: determinism and the statistics they must have."""
import math

import numpy as np

from paper_0909_0879_amd import ics


def test_plummer_deterministic_and_com():
    m1, x1, v1 = ics.plummer(1024, 1)
    m2, x2, v2 = ics.plummer(1024, 1)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    assert m1.sum() == 1.0 or abs(m1.sum() - 1.0) < 1e-15
    np.testing.assert_allclose((m1[:, None] * x1).sum(0), 0.0, atol=1e-15)
    np.testing.assert_allclose((m1[:, None] * v1).sum(0), 0.0, atol=1e-15)
    _, x3, _ = ics.plummer(1024, 2)
    assert not np.array_equal(x1, x3)


def test_plummer_mass_profile():
    # Henon-scaled Plummer: M(<r) = r^3 / (r^2 + b^2)^{3/2}
    m, x, v = ics.plummer(50000, 3)
    r = np.sort(np.linalg.norm(x, axis=1))
    b = ics.PLUMMER_HENON_B
    for q in (0.1, 0.25, 0.5, 0.75, 0.9):
        rq = r[int(q * len(r))]
        assert abs(rq ** 3 / (rq * rq + b * b) ** 1.5 - q) < 0.01


def test_plummer_kinetic_energy():
    m, x, v = ics.plummer(50000, 4)
    K = 0.5 * (m * (v * v).sum(1)).sum()
    assert abs(K - 0.25) < 0.005


def test_salpeter_mean_and_range():
    n = 200000
    u = ics.salpeter_masses(n, 3)
    assert abs(u.sum() - 1.0) < 1e-12
    raw = u * n * ics.salpeter_mean()    # undo the normalisation approximately
    assert abs(raw.mean() / ics.salpeter_mean() - 1.0) < 1e-12
    # ratio of extremes bounded by the spectrum range 0.1 .. 100
    assert u.max() / u.min() <= 1000.0 * (1 + 1e-12)
    # sample mean before normalisation ~ closed form <m> ~ 0.351
    rng = np.random.Generator(np.random.PCG64(3))
    w = rng.uniform(0.0, 1.0, n)
    p = 1.0 - ics.SALPETER_ALPHA
    mm = (0.1 ** p + w * (100.0 ** p - 0.1 ** p)) ** (1.0 / p)
    assert abs(mm.mean() / ics.salpeter_mean() - 1.0) < 0.02
    assert abs(ics.salpeter_mean() - 0.3514) < 1e-3


def test_king_profile_self_consistent():
    p = ics.king_profile(7.0)
    # concentration of a W0 = 7 King model: log10(r_t / r_0) ~ 1.53
    assert abs(math.log10(p["r_t"]) - 1.53) < 0.02
    assert np.all(np.diff(p["M"]) >= 0)
    assert p["W"][0] == 7.0 and p["W"][-1] == 0.0


def test_king_low_w0_limit_is_the_n_5_2_polytrope():
    # For small W the King density behaves as 8 W^(5/2) / (15 sqrt(pi)) times
    # (1 + 2W/7 + O(W^2)) (series of the lowered isothermal), so as W0 -> 0
    # the profile becomes the Lane-Emden n = 5/2 polytrope: with
    # r = xi sqrt(W0) / 3 the tidal radius is the polytrope's first zero
    # xi_1 = 5.35528 and M_t / (9 a^3) is its mass factor
    # -xi_1^2 theta'(xi_1) = 2.18720 (standard polytrope tables).
    c = 8.0 / (15.0 * math.sqrt(math.pi))
    for w in (1e-2, 1e-3):
        ratio = ics._king_rho(w) / (c * w ** 2.5)
        assert abs(ratio - (1.0 + 2.0 * w / 7.0)) < 2 * w * w
    w0 = 1e-4
    p = ics.king_profile(w0)
    a = math.sqrt(w0) / 3.0
    assert abs(p["r_t"] / a / 5.35528 - 1.0) < 1e-4
    assert abs(p["M_t"] / (9.0 * a ** 3) / 2.18720 - 1.0) < 1e-4
    # potential energy of an n-polytrope: -3/(5-n) G M^2 / R = -(6/5) M^2/R
    assert abs(p["pot"] / (-1.2 * p["M_t"] ** 2 / p["r_t"]) - 1.0) < 1e-3


def test_king_sample_henon_units():
    m, x, v = ics.king(20000, 7.0, 4)
    K = 0.5 * (m * (v * v).sum(1)).sum()
    assert abs(K - 0.25) < 0.01
    np.testing.assert_allclose((m[:, None] * x).sum(0), 0.0, atol=1e-14)


def test_ensemble_sizes_and_layout():
    sizes = ics.ensemble_sizes(256, 256, 16384, 5000)
    assert sizes.min() >= 256 and sizes.max() <= 16384
    assert 0.8e6 < sizes.sum() < 1.2e6
    m, x, v, off = ics.ensemble(4, sizes=[300, 512, 1000, 257], seed=5000)
    assert list(off) == [0, 300, 812, 1812, 2069]
    for c in range(4):
        sl = slice(off[c], off[c + 1])
        assert abs(m[sl].sum() - 1.0) < 1e-12
        mc, xc, vc = ics.plummer(int(off[c + 1] - off[c]), 5000 + c)
        assert np.array_equal(xc, x[sl])


def test_uniform_sphere_virial_matches_paper_setup():
    # unit mass inside the unit sphere, COM frame, K = Q |W| / 2 with the
    # continuous sphere's |W| = 3/5; the sampled W approaches -3/5
    import oracle
    m, x, v = ics.uniform_sphere_virial(2048, 11, q=1.0)
    assert abs(m.sum() - 1.0) < 1e-12
    assert np.linalg.norm(x, axis=1).max() <= 1.0 + 0.05
    assert np.abs((m[:, None] * x).sum(axis=0)).max() < 1e-12
    k = 0.5 * (m * (v * v).sum(axis=1)).sum()
    assert abs(k - 0.3) < 1e-12
    e = oracle.energy(x, v, m, 0.0)
    assert abs(e["W"] + 0.6) < 0.03
