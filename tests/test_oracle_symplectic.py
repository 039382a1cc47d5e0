"""Pins of the oracle's symplectic drivers (the paper's leapfrog and its
sixth-order explicit scheme, Sect. 4) against what the mathematics fixes:
the order conditions of the stage weights, the Kepler period and the
convergence order of each scheme, time reversibility of the symmetric
schemes, and the bounded (non-secular) energy error of a symplectic map."""
import math

import numpy as np
import pytest

import oracle


def kepler(e=0.5):
    """Two bodies of mass 1/2, semi-major axis 1 (G = 1): period 2 pi.
    Start at pericentre r = 1 - e with relative speed sqrt((1 + e) / (1 - e))."""
    r = 1.0 - e
    vrel = math.sqrt((1.0 + e) / (1.0 - e))
    x = np.array([[-r / 2, 0.0, 0.0], [r / 2, 0.0, 0.0]])
    v = np.array([[0.0, -vrel / 2, 0.0], [0.0, vrel / 2, 0.0]])
    return np.array([0.5, 0.5]), x, v


def kepler_energy(x, v):
    m = 0.5
    return 0.5 * m * (v ** 2).sum() - m * m / np.linalg.norm(x[1] - x[0])


def test_weights_satisfy_order_conditions():
    assert np.array_equal(oracle.symplectic_weights(oracle.LEAPFROG), [1.0])
    w = oracle.symplectic_weights(oracle.SYMPLECTIC6)
    assert w.shape == (7,)
    assert np.allclose(w, w[::-1], rtol=0, atol=0)          # symmetric product
    assert abs(w.sum() - 1.0) <= 1e-15
    # the third- and fifth-order error terms of a symmetric product of
    # second-order symmetric stages vanish
    assert abs((w ** 3).sum()) <= 1e-13
    assert abs((w ** 5).sum()) <= 1e-12


@pytest.mark.parametrize("scheme,n1,order", [(oracle.LEAPFROG, 2000, 2),
                                             (oracle.SYMPLECTIC6, 240, 6)])
def test_kepler_period_and_convergence_order(scheme, n1, order):
    m, x0, v0 = kepler()
    errs = []
    for n in (n1, 2 * n1):
        x, v = oracle.symplectic(x0, v0, m, 0.0, 2 * math.pi / n, n, scheme)
        errs.append(np.abs(x - x0).max())
    # after one period the orbit closes up to the truncation error
    assert errs[0] < (1e-2 if order == 2 else 1e-6)
    ratio = errs[0] / errs[1]
    assert 0.75 * 2 ** order < ratio < 1.25 * 2 ** order, (errs, ratio)


@pytest.mark.parametrize("scheme", [oracle.LEAPFROG, oracle.SYMPLECTIC6])
def test_time_reversibility(scheme):
    from paper_0909_0879_amd import ics
    m, x0, v0 = ics.plummer(64, 3)
    x, v = oracle.symplectic(x0, v0, m, 1e-2, 1 / 64, 10, scheme)
    assert np.abs(x - x0).max() > 1e-3
    x, v = oracle.symplectic(x, -v, m, 1e-2, 1 / 64, 10, scheme)
    assert np.abs(x - x0).max() <= 1e-12 * np.abs(x0).max()
    assert np.abs(-v - v0).max() <= 1e-12 * np.abs(v0).max()


@pytest.mark.parametrize("scheme,n", [(oracle.LEAPFROG, 400), (oracle.SYMPLECTIC6, 60)])
def test_energy_error_bounded(scheme, n):
    # a symplectic map conserves a nearby Hamiltonian: the energy error
    # oscillates over each orbit without a secular trend
    m, x, v = kepler()
    e0 = kepler_energy(x, v)
    h = 2 * math.pi / n
    per_orbit = []
    for orbit in range(12):
        worst = 0.0
        for _ in range(n):
            x, v = oracle.symplectic(x, v, m, 0.0, h, 1, scheme)
            worst = max(worst, abs(kepler_energy(x, v) - e0))
        per_orbit.append(worst)
    assert per_orbit[0] > 0
    assert max(per_orbit[-3:]) <= 1.5 * per_orbit[0] + 1e-14, per_orbit
