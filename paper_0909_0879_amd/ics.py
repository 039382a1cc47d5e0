"""Seeded synthetic initial conditions for the direct N-body path.

This module is the only code shared by the GPU path and the CPU oracle: it
draws particle masses, positions and velocities and holds none of the
method's arithmetic (no pairwise force, potential, predictor or corrector).
Units follow the Henon convention G = M = 1, E = -1/4; the paper takes the
total mass as the mass unit and G = 1 (Sect. 4), and Henon units are the
same convention with the length fixed by the energy instead of a radius.

Every generator takes an explicit integer seed and uses numpy's PCG64, so the
same call returns the same arrays on any machine.  All arrays are float64;
positions and velocities are (n, 3) row-major, masses (n,).

Generators
----------
plummer(n, seed)            Plummer sphere, Aarseth-Henon-Wielen (1974)
                            sampling, scaled to Henon units analytically.
salpeter_masses(n, seed)    power-law mass spectrum dN/dm ~ m^-2.35 on
                            [0.1, 100], normalised to total mass 1; the
                            paper lets masses follow a chosen spectrum
                            (Sect. 4).
king(n, w0, seed)           King (1966) lowered-isothermal model.
ensemble(n_clusters, ...)   independent Plummer clusters of log-uniform N.
uniform_sphere(n, seed)     the paper's own test set-up before the virial
                            rescale: uniform density in a unit sphere,
                            velocities uniform in direction and magnitude
                            (Sect. 4).  The rescale to a virial ratio needs
                            the potential energy, so it is left to the caller.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "plummer", "salpeter_masses", "king", "king_profile", "ensemble",
    "ensemble_sizes", "uniform_sphere", "com_frame", "isotropic",
    "PLUMMER_HENON_B", "SALPETER_ALPHA",
]

# Plummer scale length in Henon units: a Plummer sphere with G = M = b = 1
# has E = -3*pi/64; rescaling lengths to E = -1/4 gives b = 3*pi/16.
PLUMMER_HENON_B = 3.0 * math.pi / 16.0
SALPETER_ALPHA = 2.35


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors uniform on the sphere, (n, 3)."""
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def com_frame(m: np.ndarray, x: np.ndarray, v: np.ndarray):
    """Shift positions and velocities to the centre-of-mass frame."""
    mt = m.sum()
    x = x - (m[:, None] * x).sum(axis=0) / mt
    v = v - (m[:, None] * v).sum(axis=0) / mt
    return x, v


def plummer(n: int, seed: int, masses: np.ndarray | None = None,
            mass_cut: float = 0.999):
    """Plummer sphere in Henon units (G = M = 1, model energy -1/4).

    Radii from the cumulative mass fraction X ~ U(0, mass_cut):
    r = (X^(-2/3) - 1)^(-1/2) (unit scale length).  Speeds v = q * v_esc with
    v_esc = sqrt(2) (1 + r^2)^(-1/4) and q drawn by rejection from
    g(q) = q^2 (1 - q^2)^(7/2) <= 0.1 (von Neumann, bound 0.1).  Directions
    isotropic.  Lengths are then scaled by 3*pi/16 and speeds by
    sqrt(16/(3*pi)) (the analytic Henon scaling), and the system is moved to
    its centre-of-mass frame.  No per-realisation energy rescale is done:
    the sampled energy differs from -1/4 by O(N^-1/2).
    """
    if n <= 0:
        raise ValueError("n must be positive")
    rng = _rng(seed)
    m = np.full(n, 1.0 / n) if masses is None else np.asarray(masses, np.float64)
    if m.shape != (n,):
        raise ValueError("masses must have shape (n,)")
    X = rng.uniform(0.0, mass_cut, n)
    X = np.maximum(X, 1e-300)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * isotropic(rng, n)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    speed = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    v = speed[:, None] * isotropic(rng, n)
    x *= PLUMMER_HENON_B
    v *= math.sqrt(1.0 / PLUMMER_HENON_B)
    x, v = com_frame(m, x, v)
    return m, x, v


def salpeter_masses(n: int, seed: int, alpha: float = SALPETER_ALPHA,
                    m_lo: float = 0.1, m_hi: float = 100.0):
    """n masses with dN/dm ~ m^-alpha on [m_lo, m_hi] by inverse CDF, then
    normalised so that they sum to 1."""
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, n)
    p = 1.0 - alpha
    m = (m_lo ** p + u * (m_hi ** p - m_lo ** p)) ** (1.0 / p)
    return m / m.sum()


def salpeter_mean(alpha: float = SALPETER_ALPHA, m_lo: float = 0.1,
                  m_hi: float = 100.0) -> float:
    """Closed-form mean of the truncated power law (before normalisation)."""
    return ((1 - alpha) / (2 - alpha)) * (m_hi ** (2 - alpha) - m_lo ** (2 - alpha)) \
        / (m_hi ** (1 - alpha) - m_lo ** (1 - alpha))


# ---------------------------------------------------------------- King model

def _king_rho(w):
    """Dimensionless King density rho(W)/rho_1 (King 1966, lowered isothermal)."""
    w = np.maximum(np.asarray(w, np.float64), 0.0)
    from scipy.special import erf
    sw = np.sqrt(w)
    return np.exp(w) * erf(sw) - np.sqrt(4.0 * w / math.pi) * (1.0 + 2.0 * w / 3.0)


def king_profile(w0: float, npts: int = 4000):
    """Integrate the dimensionless King Poisson equation
    (1/r^2) d/dr (r^2 dW/dr) = -9 rho(W)/rho(W0), W(0) = W0, W'(0) = 0,
    out to the tidal radius where W = 0.  Radii in King core radii, with
    sigma = 1 and 4 pi G rho(W0) r0^2 / (9 sigma^2) = 1 (G = 1).

    Returns dict with r, W, M(r) (model mass units), r_t, M_t and the
    potential energy of the model, pot = -int G M(r) dM / r.
    """
    from scipy.integrate import solve_ivp
    rho0 = _king_rho(w0)

    def rhs(r, y):
        w, dw, mass = y
        rho = _king_rho(w) / rho0
        d2w = -9.0 * rho - 2.0 * dw / r
        return [dw, d2w, 9.0 * r * r * rho]   # dM/dr with 4 pi G rho0 = 9

    r_start = 1e-6
    y0 = [w0 - 1.5 * r_start ** 2, -3.0 * r_start, 3.0 * r_start ** 3]

    def hit_zero(r, y):
        return y[0]
    hit_zero.terminal = True
    hit_zero.direction = -1
    sol = solve_ivp(rhs, (r_start, 1e4), y0, events=hit_zero, rtol=1e-11,
                    atol=1e-13, dense_output=True, method="DOP853")
    r_t = float(sol.t_events[0][0])
    r = np.concatenate([[0.0], np.geomspace(r_start, r_t, npts)])
    y = sol.sol(np.clip(r, r_start, r_t))
    W = np.where(r == 0.0, w0, y[0])
    W[-1] = 0.0
    M = np.where(r == 0.0, 0.0, y[2])
    M_t = float(M[-1])
    # potential energy of the spherical model: -int_0^rt M(r) dM/dr / r dr
    rho = _king_rho(W) / rho0
    integrand = M * 9.0 * r * rho      # M(r) * (dM/dr) / r
    pot = -float(np.trapezoid(integrand, r))
    return {"r": r, "W": W, "M": M, "r_t": r_t, "M_t": M_t, "pot": pot,
            "w0": w0}


def king(n: int, w0: float, seed: int):
    """King (1966) model of n equal-mass particles in Henon units.

    Radii are drawn from the model's cumulative mass M(r) by inverse
    interpolation.  At radius r with dimensionless potential W the speed
    follows p(v) ~ v^2 (exp(W - v^2/2) - 1) on [0, sqrt(2W)] (sigma = 1),
    drawn by rejection in u = v / sqrt(2W) against a per-particle bound.
    Scaling to Henon units uses the model's own potential energy (virial
    equilibrium: E = pot/2): masses to total 1, then lengths and speeds so
    that the model energy is -1/4.  Centre-of-mass frame.
    """
    prof = king_profile(w0)
    rng = _rng(seed)
    r_tab, W_tab, M_tab = prof["r"], prof["W"], prof["M"]
    frac = M_tab / prof["M_t"]
    u = rng.uniform(0.0, 1.0, n)
    r = np.interp(u, frac, r_tab)
    W = np.maximum(np.interp(r, r_tab, W_tab), 0.0)
    x = r[:, None] * isotropic(rng, n)
    # speed by rejection: g(u) = u^2 (exp(W (1 - u^2)) - 1), u in [0, 1]
    ugrid = np.linspace(0.0, 1.0, 257)
    speed = np.empty(n)
    todo = np.arange(n)
    gmax = np.empty(n)
    for lo in range(0, n, 65536):
        w = W[lo:lo + 65536, None]
        g = ugrid[None, :] ** 2 * np.expm1(w * (1.0 - ugrid[None, :] ** 2))
        gmax[lo:lo + 65536] = g.max(axis=1) * 1.05 + 1e-300
    while todo.size:
        uu = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 1.0, todo.size) * gmax[todo]
        w = W[todo]
        ok = yy < uu * uu * np.expm1(w * (1.0 - uu * uu))
        speed[todo[ok]] = uu[ok] * np.sqrt(2.0 * w[ok])
        todo = todo[~ok]
    v = speed[:, None] * isotropic(rng, n)
    # model units -> M = 1 (G = 1): v /= sqrt(M_t); energy /= M_t^2
    M_t = prof["M_t"]
    v /= math.sqrt(M_t)
    e_model = 0.5 * prof["pot"] / (M_t * M_t)       # virial: E = W/2
    lam = e_model / (-0.25)
    x *= lam
    v /= math.sqrt(lam)
    m = np.full(n, 1.0 / n)
    x, v = com_frame(m, x, v)
    return m, x, v


# ---------------------------------------------------------------- ensemble

def ensemble_sizes(n_clusters: int, n_lo: int, n_hi: int, seed: int):
    """Cluster sizes log-uniform in [n_lo, n_hi]."""
    rng = _rng(seed)
    u = rng.uniform(math.log(n_lo), math.log(n_hi), n_clusters)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), n_lo, n_hi)


def ensemble(n_clusters: int = 256, n_lo: int = 256, n_hi: int = 16384,
             seed: int = 5000, sizes=None):
    """Independent Plummer clusters, each equal-mass in its own Henon units
    (cluster c drawn with seed + c).  Returns m, x, v concatenated and the
    int64 offsets array of length n_clusters + 1."""
    if sizes is None:
        sizes = ensemble_sizes(n_clusters, n_lo, n_hi, seed)
    sizes = np.asarray(sizes, np.int64)
    offs = np.zeros(len(sizes) + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    ms, xs, vs = [], [], []
    for c, nc in enumerate(sizes):
        m, x, v = plummer(int(nc), seed + c)
        ms.append(m)
        xs.append(x)
        vs.append(v)
    return np.concatenate(ms), np.concatenate(xs), np.concatenate(vs), offs


def uniform_sphere(n: int, seed: int, radius: float = 1.0,
                   masses: np.ndarray | None = None):
    """Uniform-density sphere with velocities uniform in direction and in
    magnitude on [0, 1] (total mass 1 unless masses are given)."""
    rng = _rng(seed)
    m = np.full(n, 1.0 / n) if masses is None else np.asarray(masses, np.float64)
    r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    x = r[:, None] * isotropic(rng, n)
    v = rng.uniform(0.0, 1.0, n)[:, None] * isotropic(rng, n)
    return m, x, v


def uniform_sphere_virial(n: int, seed: int, q: float = 1.0):
    """The initial conditions of the paper's code (Sect. 4): unit mass
    uniform in a sphere of unit radius, velocities uniform in direction and
    magnitude, rescaled to the virial ratio Q = 2K/|W|.  |W| is taken as
    the continuous uniform sphere's 3/5 (G = M = R = 1), which the sample
    approaches as N grows; the sample is shifted to its centre-of-mass frame."""
    m, x, v = uniform_sphere(n, seed)
    x = x - (m[:, None] * x).sum(axis=0) / m.sum()
    v = v - (m[:, None] * v).sum(axis=0) / m.sum()
    k = 0.5 * (m * (v * v).sum(axis=1)).sum()
    if k > 0:
        v = v * np.sqrt(0.5 * q * 0.6 / k)
    return m, x, v
