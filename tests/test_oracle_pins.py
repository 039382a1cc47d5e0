"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle's own formulas.

Force law (eq. (1) with Plummer softening): inverse-square law at a hand
computed point, shell theorem, analytic Plummer field, Newton's third law,
exact scalings and rotations, jerk = time derivative of the acceleration.
Energy (Sect. 4, virial ratio): two-body closed form and the virial
equilibrium of a Plummer sphere.  Hermite integrator and block steps (not in
the paper; motivated by the individual time steps of Sect. 3): polynomial
exactness of predictor and corrector, two-body Kepler orbit with closed-form
period and fourth-order convergence, momentum conservation, hand-built step
rules, block mode with one forced level equal to shared steps bitwise.
"""
import math

import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import ics


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- force law

def test_inverse_square_hand_value():
    # unit masses at the origin and at (3, 4, 0), eps = 0: |r| = 5,
    # a_0 = m r / |r|^3 = (3, 4, 0) / 125
    x = np.array([[0.0, 0, 0], [3.0, 4.0, 0]])
    v = np.array([[0.0, 0, 0], [0.0, 0.0, 0]])
    m = np.array([1.0, 1.0])
    a, j = oracle.forces(x, v, m, 0.0)
    np.testing.assert_allclose(a[0], [0.024, 0.032, 0.0], rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(a[1], [-0.024, -0.032, 0.0], rtol=1e-15, atol=1e-18)
    np.testing.assert_array_equal(j, 0.0)
    # softened: eps = sqrt(11) -> s = 36, s^{3/2} = 216
    a, _ = oracle.forces(x, v, m, math.sqrt(11.0))
    np.testing.assert_allclose(a[0], [3 / 216, 4 / 216, 0.0], rtol=1e-14)


def test_jerk_hand_value():
    # i at rest at origin, j of mass 2 at (1, 0, 0) moving with (0, 1, 0):
    # r.v = 0, so jerk_i = m v / r^3 = (0, 2, 0); moving along r instead,
    # v = (1, 0, 0): jerk_i = m (v - 3 (r.v) r / r^2) / r^3 = 2 (1 - 3) = -4
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    m = np.array([1.0, 2.0])
    _, j = oracle.forces(x, np.array([[0.0, 0, 0], [0.0, 1.0, 0]]), m, 0.0, idx=[0])
    np.testing.assert_allclose(j[0], [0.0, 2.0, 0.0], atol=1e-15)
    _, j = oracle.forces(x, np.array([[0.0, 0, 0], [1.0, 0.0, 0]]), m, 0.0, idx=[0])
    np.testing.assert_allclose(j[0], [-4.0, 0.0, 0.0], atol=1e-15)


def _fibonacci_shell(n, radius):
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    r = np.sqrt(1.0 - z * z)
    ph = math.pi * (1.0 + 5 ** 0.5) * k
    return radius * np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)


def test_shell_theorem():
    # a thin shell of mass 1 attracts an outside point like a point mass at
    # its centre and exerts (nearly) no force inside
    ns = 20000
    shell = _fibonacci_shell(ns, 1.0)
    probes = np.array([[3.0, 0.0, 0.0], [0.0, -2.0, 1.0], [0.3, 0.1, -0.2], [0.0, 0.0, 0.5]])
    x = np.concatenate([shell, probes])
    v = np.zeros_like(x)
    m = np.concatenate([np.full(ns, 1.0 / ns), np.zeros(len(probes))])
    idx = np.arange(ns, ns + len(probes))
    a, _ = oracle.forces(x, v, m, 0.0, idx=idx)
    for k, p in enumerate(probes):
        r = np.linalg.norm(p)
        if r > 1.0:
            want = -p / r ** 3
            assert np.linalg.norm(a[k] - want) < 2e-3 * np.linalg.norm(want)
        else:
            assert np.linalg.norm(a[k]) < 2e-3


def test_plummer_field_matches_analytic():
    # mean radial acceleration of a sampled Plummer sphere (Henon units,
    # scale length b = 3 pi/16) against -r / (r^2 + b^2)^{3/2}
    m, x, v = ics.plummer(20000, 11)
    idx = np.arange(0, 20000, 5)
    a, _ = oracle.forces(x, v, m, 1e-3, idx=idx)
    r = np.linalg.norm(x[idx], axis=1)
    ar = (a * x[idx]).sum(axis=1) / r
    b = ics.PLUMMER_HENON_B
    edges = np.quantile(r, np.linspace(0.05, 0.9, 9))
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        rm = r[sel]
        want = -(rm / (rm * rm + b * b) ** 1.5)
        got = ar[sel]
        assert abs(got.mean() / want.mean() - 1.0) < 0.04


def test_newton_third_law_pair_bitwise():
    # two equal masses: the pair terms are exact negatives of each other
    g = rng(1)
    for _ in range(20):
        x = g.normal(size=(2, 3))
        v = g.normal(size=(2, 3))
        m = np.full(2, g.uniform(0.1, 2.0))
        a, j = oracle.forces(x, v, m, g.uniform(0, 0.1))
        assert np.array_equal(a[0], -a[1])
        assert np.array_equal(j[0], -j[1])


def test_momentum_balance_small_n():
    g = rng(2)
    for n in (3, 5, 16, 64):
        x = g.normal(size=(n, 3))
        v = g.normal(size=(n, 3))
        m = g.uniform(0.1, 1.0, n)
        a, j = oracle.forces(x, v, m, 0.01)
        for q in (a, j):
            tot = np.linalg.norm((m[:, None] * q).sum(axis=0))
            scale = (m[:, None] * np.abs(q)).sum()
            assert tot <= 8 * np.finfo(float).eps * math.sqrt(n) * scale


def test_exact_transformations():
    g = rng(3)
    n = 40
    x = g.normal(size=(n, 3))
    v = g.normal(size=(n, 3))
    m = g.uniform(0.1, 1.0, n)
    a, j = oracle.forces(x, v, m, 0.02)
    # masses x 2 -> a, j x 2 exactly
    a2, j2 = oracle.forces(x, v, 2.0 * m, 0.02)
    assert np.array_equal(a2, 2 * a) and np.array_equal(j2, 2 * j)
    # reversed velocities -> jerk reversed, acceleration unchanged, exactly
    a3, j3 = oracle.forces(x, -v, m, 0.02)
    assert np.array_equal(a3, a) and np.array_equal(j3, -j)
    # rotation by 90 degrees about z: (x, y, z) -> (-y, x, z), exactly
    R = lambda q: np.stack([-q[:, 1], q[:, 0], q[:, 2]], axis=1)
    a4, j4 = oracle.forces(R(x), R(v), m, 0.02)
    assert np.array_equal(a4, R(a)) and np.array_equal(j4, R(j))
    # the self slot does not depend on the softening: one particle alone
    a5, j5 = oracle.forces(x[:1], v[:1], m[:1], 0.0)
    assert np.array_equal(a5, 0.0 * a5) and np.array_equal(j5, 0.0 * j5)


def test_jerk_is_time_derivative_of_acceleration():
    # central difference of a along straight-line motion x + v tau
    m, x, v = ics.plummer(200, 5)
    eps = 0.05
    _, j = oracle.forces(x, v, m, eps)
    errs = []
    for tau in (1e-4, 3e-5):
        ap, _ = oracle.forces(x + tau * v, v, m, eps)
        am, _ = oracle.forces(x - tau * v, v, m, eps)
        fd = (ap - am) / (2 * tau)
        errs.append((np.linalg.norm(fd - j, axis=1) / np.linalg.norm(j, axis=1)).max())
    assert errs[1] < 5e-6
    # central difference: error falls as tau^2, (10/3)^2 = 11.1
    assert 8.0 < errs[0] / errs[1] < 14.0


def test_edomain_and_einval():
    x = np.array([[0.0, 0, 0], [0.0, 0, 0]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.forces(x, np.zeros_like(x), np.ones(2), 0.0)
    assert e.value.code == oracle.EDOMAIN
    with pytest.raises(oracle.OracleError) as e:
        oracle.forces(x, np.zeros_like(x), np.ones(2), 0.0, idx=[5])
    assert e.value.code == oracle.EINVAL
    # with softening, coincident particles exert no force on each other
    a, j = oracle.forces(x, np.zeros_like(x), np.ones(2), 0.1)
    assert np.array_equal(a, np.zeros_like(a))


def test_potential_hand_value():
    x = np.array([[0.0, 0, 0], [3.0, 4.0, 0]])
    m = np.array([1.0, 2.0])
    a, j, pot = oracle.forces(x, np.zeros_like(x), m, 0.0, want_pot=True)
    np.testing.assert_allclose(pot, [-2.0 / 5.0, -1.0 / 5.0], rtol=1e-15)


# ---------------------------------------------------------------- energy

def test_energy_two_body_hand_value():
    # m = 1/2 each at distance 1, velocities +-(0, 1/2, 0):
    # K = 2 * 1/2 * 1/2 * 1/4 = 1/8, W = -1/4, L_z = 2 * 1/2 * 1/2 * 1/2 = 1/4
    x = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v = np.array([[0, -0.5, 0], [0, 0.5, 0]])
    e = oracle.energy(x, v, np.array([0.5, 0.5]), 0.0)
    assert e["K"] == 0.125 and e["W"] == -0.25 and e["E"] == -0.125
    np.testing.assert_array_equal(e["L"], [0, 0, 0.25])
    np.testing.assert_array_equal(e["P"], [0, 0, 0])


def test_plummer_virial_equilibrium():
    # Henon units: W = -1/2, K = 1/4, virial ratio Q = 2K/|W| = 1 (Sect. 4)
    m, x, v = ics.plummer(8192, 7)
    e = oracle.energy(x, v, m, 1e-4)
    assert abs(e["W"] + 0.5) < 0.03
    assert abs(e["K"] - 0.25) < 0.015
    assert abs(2 * e["K"] / abs(e["W"]) - 1.0) < 0.05
    np.testing.assert_allclose(e["P"], 0.0, atol=1e-15)


# ---------------------------------------------------------------- Hermite

def test_predictor_exact_for_constant_jerk():
    g = rng(4)
    for _ in range(10):
        x0, v0, a0, j0 = (g.normal(size=3) for _ in range(4))
        dt = 2.0 ** -g.integers(1, 8)
        xp, vp = oracle.predict_one(x0, v0, a0, j0, dt)
        np.testing.assert_allclose(xp, x0 + v0 * dt + a0 * dt ** 2 / 2 + j0 * dt ** 3 / 6,
                                   rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(vp, v0 + a0 * dt + j0 * dt ** 2 / 2, rtol=1e-14, atol=1e-15)


def test_corrector_exact_for_cubic_acceleration():
    # a(t) = A0 + A1 t + A2 t^2/2 + A3 t^3/6 is reproduced exactly by the
    # fourth-order Hermite corrector, so x(h), v(h) come out exact
    g = rng(5)
    for _ in range(10):
        x0, v0, A0, A1, A2, A3 = (g.normal(size=3) for _ in range(6))
        h = 2.0 ** -g.integers(1, 6)
        a1 = A0 + A1 * h + A2 * h ** 2 / 2 + A3 * h ** 3 / 6
        j1 = A1 + A2 * h + A3 * h ** 2 / 2
        xp, vp = oracle.predict_one(x0, v0, A0, A1, h)
        x1, v1, a2e, a3 = oracle.correct_one(xp, vp, A0, A1, a1, j1, h)
        xe = x0 + v0 * h + A0 * h ** 2 / 2 + A1 * h ** 3 / 6 + A2 * h ** 4 / 24 + A3 * h ** 5 / 120
        ve = v0 + A0 * h + A1 * h ** 2 / 2 + A2 * h ** 3 / 6 + A3 * h ** 4 / 24
        np.testing.assert_allclose(x1, xe, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(v1, ve, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(a2e, A2 + A3 * h, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(a3, A3, rtol=1e-8, atol=1e-8)


def test_aarseth_criterion_hand_value():
    # |a| = 1, |j| = 1, |a2| = 2, |a3| = 0: dt = sqrt(eta (1*2 + 1) / (0 + 4))
    dt = oracle.aarseth_dt([1, 0, 0], [0, 1, 0], [0, 0, 2], [0, 0, 0], 0.01)
    assert dt == pytest.approx(math.sqrt(0.0075), rel=1e-15)
    # |a| = 2, |j| = 3, |a2| = 0, |a3| = 4: sqrt(eta * 9 / 12)
    dt = oracle.aarseth_dt([2, 0, 0], [0, 3, 0], [0, 0, 0], [0, 4, 0], 0.02)
    assert dt == pytest.approx(math.sqrt(0.015), rel=1e-15)
    assert oracle.aarseth_dt([1, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], 0.01) == math.inf


def test_block_level_rules():
    T = 1 << 20
    # halving until <= dt_c: dt = 1/32, dt_c = 0.01 -> 1/128
    assert oracle.next_level(5, 0.01, T // 32, 3, 20) == (7, 0)
    # doubling allowed only at a multiple of the doubled step
    assert oracle.next_level(5, 0.1, 2 * (T // 32), 3, 20) == (4, 0)
    assert oracle.next_level(5, 0.1, 3 * (T // 32), 3, 20) == (5, 0)
    # doubling needs dt_c >= 2 dt
    assert oracle.next_level(5, 0.06, 2 * (T // 32), 3, 20) == (5, 0)
    # never above dt_max = 2^-level_min
    assert oracle.next_level(3, 10.0, 0, 3, 20) == (3, 0)
    # floor clamp counted
    assert oracle.next_level(18, 1e-9, 0, 3, 20) == (20, 1)
    # dt_c exactly equal to the step keeps it
    assert oracle.next_level(6, 2.0 ** -6, T // 64, 3, 20) == (6, 0)
    # initial level: eta |a|/|j| = 0.01 * 1 / 2 = 0.005 -> 2^-8
    assert oracle.initial_level([1, 0, 0], [0, 0, 2], 0.01, 3, 20) == (8, 0)
    assert oracle.initial_level([1, 0, 0], [0, 0, 0], 0.01, 3, 20) == (3, 0)
    assert oracle.initial_level([1e-12, 0, 0], [0, 0, 1], 0.01, 3, 20) == (20, 1)


def _kepler(e=0.5):
    # m1 = m2 = 1/2 (M = 1), semi-major axis 1, start at pericentre
    rp = 1 - e
    vp = math.sqrt((1 + e) / (1 - e))
    m = np.array([0.5, 0.5])
    x = np.array([[-rp / 2, 0, 0], [rp / 2, 0, 0]])
    v = np.array([[0, -vp / 2, 0], [0, vp / 2, 0]])
    return m, x, v


def _kepler_separation(t, e=0.5):
    # closed form: period 2 pi, mean motion 1; solve E - e sin E = t
    E = t
    for _ in range(60):
        E -= (E - e * math.sin(E) - t) / (1 - e * math.cos(E))
    return np.array([math.cos(E) - e, math.sqrt(1 - e * e) * math.sin(E), 0.0])


def _kepler_run(level):
    dt = 2.0 ** -level
    m, x, v = _kepler()
    s = oracle.System(m, x, v, 0.0, dt_shared=dt, level_min=level, level_max=level)
    e0 = s.energy()
    T = round(2 * math.pi / dt) * dt
    s.run(T)
    err = np.linalg.norm((s.x[1] - s.x[0]) - _kepler_separation(T))
    e1 = s.energy()
    return s, e0, e1, err


def test_kepler_orbit_period_and_convergence():
    errs = []
    for level in (7, 8, 9):
        s, e0, e1, err = _kepler_run(level)
        errs.append(err)
        de = abs(e1["E"] - e0["E"]) / abs(e0["E"])
        assert de < 1e-8
        # conserved: total momentum exactly (shared steps), angular momentum
        np.testing.assert_allclose(e1["P"], 0.0, atol=1e-15)
        assert abs(e1["L"][2] - e0["L"][2]) / e0["L"][2] < 1e-7
        # semi-major axis and eccentricity from E and L (reduced mass 1/4)
        mu, k = 0.25, 0.25                        # reduced mass, G m1 m2
        a_orb = -k / (2 * e1["E"])
        ecc = math.sqrt(1 + 2 * e1["E"] * e1["L"][2] ** 2 / (mu * k * k))
        assert abs(a_orb - 1.0) < 1e-7
        assert abs(ecc - 0.5) < 1e-6
    assert errs[0] < 1e-5
    for r in (errs[0] / errs[1], errs[1] / errs[2]):
        assert 12.0 < r < 20.0          # fourth order: dt/2 -> error / 16


def test_block_mode_single_level_equals_shared_bitwise():
    m, x, v = ics.plummer(128, 9)
    s1 = oracle.System(m, x, v, 1e-2, dt_shared=2.0 ** -7, level_min=7, level_max=7)
    s2 = oracle.System(m, x, v, 1e-2, dt_shared=0.0, level_min=7, level_max=7)
    s1.run(2.0 ** -3)
    s2.run(2.0 ** -3)
    assert np.array_equal(s1.x, s2.x) and np.array_equal(s1.v, s2.v)
    assert np.array_equal(s1.a, s2.a) and np.array_equal(s1.j, s2.j)
    assert s1.stats.n_block_steps == s2.stats.n_block_steps == 16


def test_block_steps_invariants():
    m, x, v = ics.plummer(256, 10)
    s = oracle.System(m, x, v, 1e-2, eta=0.02, eta_start=0.01, level_min=3, level_max=20)
    e0 = s.energy()
    s.run(0.125)
    assert (s.tick == (1 << 17)).all()          # everyone synchronised at t_end
    lv = s.level.astype(np.int64)
    assert (lv >= 3).all() and (lv <= 20).all()
    assert len(np.unique(lv)) > 1                # block steps really used
    assert s.stats.n_interactions < s.stats.n_block_steps * 256 * 256
    e1 = s.energy()
    assert abs(e1["E"] - e0["E"]) / abs(e0["E"]) < 1e-5
    # block steps update particles at different times: momentum is kept to
    # the integration error, not to rounding
    assert np.linalg.norm(e1["P"]) < 1e-7 * (m * np.linalg.norm(v, axis=1)).sum()


def test_shared_step_momentum_exact():
    m, x, v = ics.plummer(64, 12)
    s = oracle.System(m, x, v, 1e-2, dt_shared=2.0 ** -8, level_min=8, level_max=8)
    p0 = s.energy()["P"]
    s.run(2.0 ** -4)
    assert np.linalg.norm(s.energy()["P"] - p0) < 1e-15


def test_block_step_energy_drift_shrinks_with_eta():
    # the Hermite scheme is fourth order, so halving the accuracy parameter
    # eta (step ~ eta) should cut the energy error by about 2^4; close
    # encounters make single runs noisy, so the sum over four Plummer
    # spheres is compared, with a factor 4 of margin
    drift = {}
    for eta in (0.02, 0.01):
        tot = 0.0
        for seed in (21, 22, 23, 24):
            m, x, v = ics.plummer(2048, seed)
            s = oracle.System(m, x, v, 1e-3, eta=eta, eta_start=eta, level_min=4,
                              level_max=20)
            e0 = s.energy()["E"]
            s.run(1 / 16)
            tot += abs(s.energy()["E"] - e0) / abs(e0)
        drift[eta] = tot
    assert drift[0.01] * 4 < drift[0.02], drift
