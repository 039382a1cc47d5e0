"""Pins of the oracle's external Galactic field (the Allen & Santillan 1991
model the paper adds to the pairwise forces, Sect. 4) and of its coupling
into the oracle's integrators and energy, against what the literature and
the mathematics fix: the model's published circular velocity at the Sun and
total mass, acc = -grad Phi and jerk = d acc / dt by central differences,
the Miyamoto-Nagai disk with a = 0 reducing to a Plummer sphere, the halo's
point-mass exterior, and a circular orbit held by the Hermite and
symplectic drivers with energy and L_z conserved."""
import math
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
FIELD_KEYS = oracle.FIELD_KEYS


def model():
    vals = {}
    with open(os.path.join(HERE, "golden", "allen_santillan_1991.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    field = {k: vals[k] for k in FIELD_KEYS}
    return field, vals


def v_unit_kms(vals):
    # velocity unit of the model: sqrt(G * mass unit / 1 kpc)
    return math.sqrt(vals["g_kpc_kms2_msun"] * vals["mass_unit_msun"])


def test_circular_velocity_at_sun():
    field, vals = model()
    R = vals["r_sun_kpc"]
    acc, _, _ = oracle.field_eval(field, [R, 0.0, 0.0], [0.0, 0.0, 0.0])
    assert acc[0] < 0 and acc[1] == 0 and acc[2] == 0
    vc = math.sqrt(R * -acc[0]) * v_unit_kms(vals)
    assert abs(vc - vals["v_circ_sun_kms"]) <= 0.005 * vals["v_circ_sun_kms"], vc


def test_total_mass_by_gauss_theorem():
    # flux of the field through the sphere r = r_c: -(r^2 / 2) int a_r sin(t) dt
    field, vals = model()
    r = vals["halo_rc"]
    mu, w = np.polynomial.legendre.leggauss(96)        # mu = cos(theta)
    st = np.sqrt(1 - mu * mu)
    pts = np.stack([r * st, np.zeros_like(mu), r * mu], axis=1)
    acc, _, _ = oracle.field_eval(field, pts, np.zeros_like(pts))
    a_r = np.sum(acc * pts, axis=1) / r
    m_enc = -(r * r / 2) * np.sum(w * a_r)
    m_sun = m_enc * vals["mass_unit_msun"]
    assert abs(m_sun - vals["m_total_msun"]) <= 0.02 * vals["m_total_msun"], m_sun


def _points(rng, n):
    # spread over the disk plane, the bulge, the halo and beyond the cut-off
    r = np.exp(rng.uniform(np.log(0.05), np.log(300.0), n))
    mu = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - mu * mu)
    x = np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * mu], axis=1)
    x[: n // 4, 2] *= 0.01                            # near the midplane
    v = rng.normal(size=(n, 3)) * 20.0
    return x, v


def test_acceleration_is_minus_gradient_of_potential():
    field, _ = model()
    rng = np.random.default_rng(1)
    x, v = _points(rng, 200)
    acc, _, _ = oracle.field_eval(field, x, v)
    for i in range(x.shape[0]):
        h = 1e-5 * max(np.linalg.norm(x[i]), 1e-2)
        grad = np.empty(3)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            pp = oracle.field_eval(field, x[i] + e, v[i])[2]
            pm = oracle.field_eval(field, x[i] - e, v[i])[2]
            grad[c] = (pp - pm) / (2 * h)
        assert np.linalg.norm(acc[i] + grad) <= 1e-6 * np.linalg.norm(acc[i]), (x[i], acc[i], grad)


def test_jerk_is_time_derivative_of_acceleration():
    field, _ = model()
    rng = np.random.default_rng(2)
    x, v = _points(rng, 200)
    _, jerk, _ = oracle.field_eval(field, x, v)
    for i in range(x.shape[0]):
        h = 1e-5 * max(np.linalg.norm(x[i]), 1e-2) / np.linalg.norm(v[i])
        ap = oracle.field_eval(field, x[i] + h * v[i], v[i])[0]
        am = oracle.field_eval(field, x[i] - h * v[i], v[i])[0]
        fd = (ap - am) / (2 * h)
        assert np.linalg.norm(jerk[i] - fd) <= 1e-6 * np.linalg.norm(jerk[i]) + 1e-12, i


def test_each_component_alone():
    # every component is pinned by the same two identities on its own, so a
    # slip in one cannot hide behind the others
    field, _ = model()
    rng = np.random.default_rng(3)
    x, v = _points(rng, 40)
    for keys in (("bulge_m", "bulge_b"), ("disk_m", "disk_a", "disk_b"),
                 ("halo_m", "halo_a", "halo_gamma", "halo_rc")):
        f = {k: field[k] for k in keys}
        if "halo_m" not in f:
            f.update(halo_a=1.0, halo_gamma=1.0, halo_rc=1.0)
        acc, jerk, _ = oracle.field_eval(f, x, v)
        assert np.all(np.isfinite(acc)) and np.any(acc != 0), keys
        for i in range(x.shape[0]):
            h = 1e-5 * max(np.linalg.norm(x[i]), 1e-2)
            grad = np.array([(oracle.field_eval(f, x[i] + h * e, v[i])[2]
                              - oracle.field_eval(f, x[i] - h * e, v[i])[2]) / (2 * h)
                             for e in np.eye(3)])
            assert np.linalg.norm(acc[i] + grad) <= 1e-6 * np.linalg.norm(acc[i]), keys
            ht = h / np.linalg.norm(v[i])
            fd = (oracle.field_eval(f, x[i] + ht * v[i], v[i])[0]
                  - oracle.field_eval(f, x[i] - ht * v[i], v[i])[0]) / (2 * ht)
            assert np.linalg.norm(jerk[i] - fd) <= 1e-6 * np.linalg.norm(jerk[i]) + 1e-12, keys


def test_disk_with_zero_radial_scale_is_plummer_sphere():
    rng = np.random.default_rng(4)
    x, v = _points(rng, 50)
    disk = oracle.field_eval({"disk_m": 3.0, "disk_a": 0.0, "disk_b": 0.7}, x, v)
    bulge = oracle.field_eval({"bulge_m": 3.0, "bulge_b": 0.7}, x, v)
    for d, b in zip(disk, bulge):
        assert np.allclose(d, b, rtol=1e-13, atol=0)


def test_plummer_bulge_closed_form():
    # on the axis the Plummer potential and pull are textbook values
    r, M, b = 2.0, 5.0, 0.5
    acc, _, pot = oracle.field_eval({"bulge_m": M, "bulge_b": b}, [0, 0, r], [0, 0, 0])
    assert math.isclose(pot, -M / math.sqrt(r * r + b * b), rel_tol=1e-15)
    assert math.isclose(acc[2], -M * r / (r * r + b * b) ** 1.5, rel_tol=1e-15)


def test_halo_exterior_is_point_mass_and_continuous():
    field, vals = model()
    halo = {k: field[k] for k in ("halo_m", "halo_a", "halo_gamma", "halo_rc")}
    rc = halo["halo_rc"]
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    # beyond r_c: r^2 |a| and r * Phi are the same constant (the enclosed mass)
    outs = [oracle.field_eval(halo, r * d, np.zeros(3)) for r in (1.2 * rc, 2 * rc, 7 * rc)]
    m_enc = [np.linalg.norm(a) * r * r for (a, _, _), r in zip(outs, (1.2 * rc, 2 * rc, 7 * rc))]
    m_pot = [-p * r for (_, _, p), r in zip(outs, (1.2 * rc, 2 * rc, 7 * rc))]
    assert np.allclose(m_enc, m_enc[0], rtol=1e-14) and np.allclose(m_pot, m_enc[0], rtol=1e-14)
    # the potential and the pull are continuous across r_c
    lo = oracle.field_eval(halo, rc * (1 - 1e-9) * d, np.zeros(3))
    hi = oracle.field_eval(halo, rc * (1 + 1e-9) * d, np.zeros(3))
    assert abs(lo[2] - hi[2]) <= 1e-8 * abs(hi[2])
    assert np.linalg.norm(lo[0] - hi[0]) <= 1e-8 * np.linalg.norm(hi[0])
    # inside, r^2 |a| grows with r (mass keeps being enclosed)
    inner = [np.linalg.norm(oracle.field_eval(halo, r * d, np.zeros(3))[0]) * r * r
             for r in (1.0, 10.0, 50.0, 99.0)]
    assert np.all(np.diff(inner) > 0) and inner[-1] < m_enc[0]
    # at the centre the halo adds nothing
    a0, j0, _ = oracle.field_eval(halo, np.zeros(3), np.ones(3))
    assert np.all(a0 == 0) and np.all(j0 == 0)


def _circular(field, R):
    acc, _, _ = oracle.field_eval(field, [R, 0.0, 0.0], [0.0, 0.0, 0.0])
    vc = math.sqrt(R * -acc[0])
    m = np.array([1e-12])
    x = np.array([[R, 0.0, 0.0]])
    v = np.array([[0.0, vc, 0.0]])
    return m, x, v, vc


def test_hermite_is_fourth_order_on_circular_orbit():
    # shared steps 2^-5 ... 2^-7 over about one orbit: the distance to the
    # exact circular orbit falls 16 times per halving (a wrong field jerk
    # would break the corrector's a2, a3 and lower the order)
    field, vals = model()
    R = vals["r_sun_kpc"]
    m, x, v, vc = _circular(field, R)
    om, t = vc / R, 2.5                    # 2 pi R / v_c = 2.43
    x_exact = R * np.array([math.cos(om * t), math.sin(om * t), 0.0])
    err = []
    for lv in (5, 6, 7):
        s = oracle.System(m, x, v, 0.0, dt_shared=2.0 ** -lv, level_min=1, level_max=20,
                          field=field)
        e0 = s.energy()
        s.run(t)
        e1 = s.energy()
        err.append(np.linalg.norm(s.x[0] - x_exact))
    assert 12 <= err[0] / err[1] <= 22 and 12 <= err[1] / err[2] <= 22, err
    assert err[2] <= 1e-6 * R
    assert abs(e1["E"] - e0["E"]) <= 1e-9 * abs(e0["E"])
    assert abs(e1["L"][2] - e0["L"][2]) <= 1e-9 * abs(e0["L"][2])
    # the energy holds the field's potential energy
    pot = oracle.field_eval(field, s.x[0], s.v[0])[2]
    assert math.isclose(e1["E"] - e1["K"] - e1["W"], m[0] * pot, rel_tol=1e-12)


def test_hermite_block_steps_keep_circular_orbit():
    field, vals = model()
    R = vals["r_sun_kpc"]
    m, x, v, vc = _circular(field, R)
    s = oracle.System(m, x, v, 0.0, eta=0.01, eta_start=0.01, level_min=1, level_max=20,
                      field=field)
    e0 = s.energy()
    s.run(2.5)
    assert abs(np.linalg.norm(s.x[0]) - R) <= 1e-5 * R
    assert abs(s.energy()["E"] - e0["E"]) <= 1e-6 * abs(e0["E"])


def test_symplectic_orders_on_circular_orbit():
    # after one period the leapfrog's error falls 4 times per halving of h,
    # the sixth-order scheme's 64 times
    field, vals = model()
    R = vals["r_sun_kpc"]
    m, x, v, vc = _circular(field, R)
    period = 2 * math.pi * R / vc
    for scheme, lo, hi in ((oracle.LEAPFROG, 3.5, 4.5), (oracle.SYMPLECTIC6, 45, 85)):
        err = []
        for n in (128, 256):
            xs, _ = oracle.symplectic(x, v, m, 0.0, period / n, n, scheme, field=field)
            err.append(np.linalg.norm(xs[0] - x[0]))
        assert lo <= err[0] / err[1] <= hi, (scheme, err)


def test_cluster_in_field_conserves_energy():
    # a small Plummer cluster on a circular Galactic orbit (cluster units:
    # 1e5 M_sun, 1 pc), Hermite block steps with the field
    from paper_0909_0879_amd import ics
    field, vals = model()
    mass_msun, length_kpc = 1e5, 1e-3
    f = {k: field[k] * vals["mass_unit_msun"] / mass_msun if k.endswith("_m")
         else (field[k] if k == "halo_gamma" else field[k] / length_kpc) for k in FIELD_KEYS}
    R = vals["r_sun_kpc"] / length_kpc
    m, x, v = ics.plummer(128, 5)
    _, _, _, vc = _circular(f, R)
    x = x + np.array([R, 0.0, 0.0])
    v = v + np.array([0.0, vc, 0.0])
    t = 0.5
    s = oracle.System(m, x, v, 1e-2, eta=0.01, eta_start=0.01, level_min=3, level_max=20,
                      field=f)
    e0 = s.energy()
    s.run(t)
    e1 = s.energy()
    # conserved to a small fraction of the cluster's own binding energy
    assert abs(e1["E"] - e0["E"]) <= 1e-7 * abs(e0["W"])
    assert abs(e1["L"][2] - e0["L"][2]) <= 1e-9 * abs(e0["L"][2])
    # the field pulls the centre of mass inwards by a_c t^2 / 2 (a_c = v_c^2 / R)
    # relative to the same cluster without it
    free = oracle.System(m, x, v, 1e-2, eta=0.01, eta_start=0.01, level_min=3, level_max=20)
    free.run(t)
    dx = (m @ s.x - m @ free.x) / m.sum()
    assert abs(dx[0] + 0.5 * vc * vc / R * t * t) <= 0.01 * 0.5 * vc * vc / R * t * t, dx
