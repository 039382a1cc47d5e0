/*
 * Plain FP64 CPU oracle for the direct N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library.  It shares
 * no code, header, table or helper with the GPU library; it is written for
 * a reader checking it against the paper, not for speed.
 *
 * What is computed (G = 1, Sect. 4 of the paper):
 *   r_ij = x_j - x_i,  v_ij = v_j - v_i,  s_ij = |r_ij|^2 + eps^2
 *   a_i  = sum_{j != i} m_j r_ij s_ij^{-3/2}                     eq. (1)
 *   j_i  = sum_{j != i} m_j [ v_ij s^{-3/2} - 3 (r_ij.v_ij) r_ij s^{-5/2} ]
 *   phi_i = -sum_{j != i} m_j s_ij^{-1/2}
 * Eq. (1) is the unsoftened acceleration; the paper adds a softening length
 * eps to the pair potential (Sect. 4) without giving its form, read here as
 * the Plummer form phi = -m / sqrt(r^2 + eps^2).  The jerk is the time
 * derivative of a_i along the current velocities (not in the paper).
 *
 * External field (Sect. 4): the pairwise forces are added to the force of
 * an analytic Galactic potential, the three-component model of Allen &
 * Santillan (1991) the paper names (spherical bulge, axisymmetric disk,
 * spherical halo).  The paper prints neither the formulas nor the
 * parameters; the forms used are given at oracle_field_eval, and the
 * published parameters are supplied by the caller.
 *
 * Time integration: the paper's symplectic drivers (leapfrog and a
 * sixth-order composition of leapfrog stages, Sect. 4) for shared steps,
 * and a fourth-order Hermite predictor-corrector (Makino &
 * Aarseth 1992 form) with individual, power-of-two block time steps chosen
 * by Aarseth's criterion.  The paper motivates individual per-particle steps
 * and the care they need for synchronisation (Sect. 3); the integrator
 * itself is not in the paper.  Times are integer ticks of 2^-20.
 *
 * Sums are Neumaier-compensated so that the oracle is more accurate than
 * either GPU path; j runs in ascending order and skips j == i.  OpenMP runs
 * over i only, so results do not depend on the thread count.
 *
 * Parity pins for each function are listed with it; see the tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENONFINITE -6
#define OR_EDOMAIN -7

#define OR_TICK_BITS 20          /* one time unit = 2^20 ticks */
#define OR_MAX_LEVEL 20

/* ---------------------------------------------------------------- sums */

/* Neumaier's improved Kahan-Babuska summation: (s, c) holds sum + error. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_val(const nsum *a) { return a->s + a->c; }

/* ---------------------------------------------------------------- forces */

/* Pair sum for one i over j in [0, n_j), skipping j == self (eq. (1) with
 * Plummer softening, plus jerk and potential).  Returns OR_EDOMAIN when
 * eps == 0 and a distinct j sits exactly on i (the sum is undefined). */
static int force_one(int64_t self, const double xi[3], const double vi[3],
                     int64_t n_j, const double *x, const double *v,
                     const double *m, double eps, double acc[3],
                     double jerk[3], double *pot) {
  nsum sa[3], sj[3], sp;
  memset(sa, 0, sizeof sa);
  memset(sj, 0, sizeof sj);
  memset(&sp, 0, sizeof sp);
  const double eps2 = eps * eps;
  for (int64_t j = 0; j < n_j; ++j) {
    if (j == self) continue;
    const double rx = x[3 * j + 0] - xi[0];
    const double ry = x[3 * j + 1] - xi[1];
    const double rz = x[3 * j + 2] - xi[2];
    const double wx = v[3 * j + 0] - vi[0];
    const double wy = v[3 * j + 1] - vi[1];
    const double wz = v[3 * j + 2] - vi[2];
    const double s = rx * rx + ry * ry + rz * rz + eps2;
    if (s == 0.0) return OR_EDOMAIN;
    const double rinv = 1.0 / sqrt(s);          /* s^{-1/2}, IEEE sqrt and divide */
    const double rinv2 = rinv * rinv;           /* s^{-1}   */
    const double mr3 = m[j] * rinv * rinv2;     /* m s^{-3/2} */
    const double rv = rx * wx + ry * wy + rz * wz;
    const double alpha = 3.0 * rv * rinv2;      /* 3 (r.v) / s */
    nsum_add(&sa[0], mr3 * rx);
    nsum_add(&sa[1], mr3 * ry);
    nsum_add(&sa[2], mr3 * rz);
    nsum_add(&sj[0], mr3 * (wx - alpha * rx));
    nsum_add(&sj[1], mr3 * (wy - alpha * ry));
    nsum_add(&sj[2], mr3 * (wz - alpha * rz));
    nsum_add(&sp, -m[j] * rinv);
  }
  for (int c = 0; c < 3; ++c) {
    acc[c] = nsum_val(&sa[c]);
    jerk[c] = nsum_val(&sj[c]);
  }
  *pot = nsum_val(&sp);
  return OR_OK;
}

/* Acceleration, jerk and potential on particles idx[0..n_i) of a set of n_j
 * particles (positions x, velocities v, (n_j, 3) row-major; masses m).  The
 * i-particle's own slot is skipped; idx may repeat.  acc, jerk: (n_i, 3);
 * pot: (n_i) or NULL.  Pins: brute-force Newton-III antisymmetry, closed
 * two-body values, jerk = finite difference of acc, shell theorem, the
 * analytic Plummer field, exact mass/velocity/axis transformations. */
int oracle_forces(int64_t n_i, const int64_t *idx, int64_t n_j,
                  const double *x, const double *v, const double *m,
                  double eps, double *acc, double *jerk, double *pot) {
  if (n_i < 0 || n_j < 0 || eps < 0.0) return OR_EINVAL;
  int err = OR_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n_i; ++k) {
    const int64_t i = idx[k];
    double p = 0.0;
    if (i < 0 || i >= n_j) {
#pragma omp atomic write
      err = OR_EINVAL;
      continue;
    }
    int e = force_one(i, &x[3 * i], &v[3 * i], n_j, x, v, m, eps,
                      &acc[3 * k], &jerk[3 * k], &p);
    if (e) {
#pragma omp atomic write
      err = e;
    }
    if (pot) pot[k] = p;
  }
  return err;
}

/* --------------------------------------------------------- external field */

/* Parameters of the three components, G = 1 in the caller's units; a zero
 * mass switches a component off. */
typedef struct {
  double bulge_m, bulge_b;            /* bulge mass and scale length */
  double disk_m, disk_a, disk_b;      /* disk mass, radial and vertical scales */
  double halo_m, halo_a, halo_gamma;  /* halo mass scale, radius, exponent */
  double halo_rc;                     /* halo cut-off radius */
} oracle_field;

/* Spherical component: acc = -g(r) x, jerk = -(g v + (g'(r) / r) (x.v) x),
 * the time derivative of the acceleration along v. */
static void sph_add(double g, double gp_over_r, const double x[3],
                    const double v[3], double acc[3], double jerk[3]) {
  const double xv = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
  for (int c = 0; c < 3; ++c) {
    acc[c] -= g * x[c];
    jerk[c] -= g * v[c] + gp_over_r * xv * x[c];
  }
}

/* The external field at position x moving with velocity v:
 *   bulge (Plummer sphere): Phi = -M / sqrt(r^2 + b^2), so
 *     g = M (r^2 + b^2)^(-3/2), g'/r = -3 M (r^2 + b^2)^(-5/2).
 *   disk (Miyamoto & Nagai 1975): zeta = sqrt(z^2 + b^2), u = a + zeta,
 *     D = sqrt(R^2 + u^2), Phi = -M / D;
 *     acc = -M (x, y, z u / zeta) / D^3; with q = x vx + y vy + u z vz / zeta
 *     (= D dD/dt) and d(z u / zeta)/dt = vz (u b^2 / zeta^3 + z^2 / zeta^2),
 *     jerk = -M [ (vx, vy, vz (u b^2 / zeta^3 + z^2 / zeta^2)) / D^3
 *                 - 3 q (x, y, z u / zeta) / D^5 ].
 *   halo: enclosed mass M(r) = M_h s^(g+1) / (1 + s^g), s = r / a, up to
 *     r_c and M(r_c) beyond; force -M(r) / r^2 radially, i.e.
 *     g(r) = M(r) / r^3, g'/r = M'(r) / r^4 - 3 M(r) / r^5 with
 *     M'(r) = (M_h / a) s^g (g + 1 + s^g) / (1 + s^g)^2 inside, 0 beyond;
 *     potential the integral of that force from infinity:
 *     Phi = -M(r_c) / r beyond r_c,
 *     Phi = -M(r_c) / r_c - (M_h / (g a)) [ln(1 + s_c^g) - ln(1 + s^g)] inside.
 *     At r = 0 the halo adds nothing (its acceleration tends to zero there).
 * pot receives Phi (per unit mass).  Pins: the published circular velocity
 * at the Sun and total mass of the model, acc = -grad Phi and jerk = d acc /
 * dt by central differences, the disk with a = 0 equal to the Plummer
 * bulge, the halo continuous at r_c and a point mass beyond, a circular
 * orbit kept by the Hermite driver. */
void oracle_field_eval(const oracle_field *f, const double x[3], const double v[3],
                       double acc[3], double jerk[3], double *pot) {
  double phi = 0.0;
  for (int c = 0; c < 3; ++c) acc[c] = jerk[c] = 0.0;
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  if (f->bulge_m != 0.0) {
    const double d2 = r2 + f->bulge_b * f->bulge_b;
    const double d = sqrt(d2);
    const double g = f->bulge_m / (d2 * d);
    sph_add(g, -3.0 * g / d2, x, v, acc, jerk);
    phi -= f->bulge_m / d;
  }
  if (f->disk_m != 0.0) {
    const double M = f->disk_m, b = f->disk_b;
    const double z = x[2];
    const double zeta = sqrt(z * z + b * b);
    const double u = f->disk_a + zeta;
    const double D2 = x[0] * x[0] + x[1] * x[1] + u * u;
    const double D = sqrt(D2);
    const double D3 = D2 * D, D5 = D3 * D2;
    const double zf = z * u / zeta;
    const double q = x[0] * v[0] + x[1] * v[1] + v[2] * zf;
    const double dzf = v[2] * (u * b * b / (zeta * zeta * zeta) + z * z / (zeta * zeta));
    acc[0] -= M * x[0] / D3;
    acc[1] -= M * x[1] / D3;
    acc[2] -= M * zf / D3;
    jerk[0] -= M * (v[0] / D3 - 3.0 * q * x[0] / D5);
    jerk[1] -= M * (v[1] / D3 - 3.0 * q * x[1] / D5);
    jerk[2] -= M * (dzf / D3 - 3.0 * q * zf / D5);
    phi -= M / D;
  }
  if (f->halo_m != 0.0 && r2 > 0.0) {
    const double a = f->halo_a, gm = f->halo_gamma, Mh = f->halo_m;
    const double r = sqrt(r2);
    const double sc = f->halo_rc / a;
    const double scg = pow(sc, gm);
    const double Mc = Mh * sc * scg / (1.0 + scg);    /* M(r_c) */
    double Mr, Mp;
    if (r < f->halo_rc) {
      const double s = r / a, sg = pow(s, gm);
      Mr = Mh * s * sg / (1.0 + sg);
      Mp = (Mh / a) * sg * (gm + 1.0 + sg) / ((1.0 + sg) * (1.0 + sg));
      phi += -Mc / f->halo_rc - (Mh / (gm * a)) * (log(1.0 + scg) - log(1.0 + sg));
    } else {
      Mr = Mc;
      Mp = 0.0;
      phi -= Mc / r;
    }
    const double r3 = r2 * r;
    sph_add(Mr / r3, Mp / (r3 * r) - 3.0 * Mr / (r3 * r2), x, v, acc, jerk);
  }
  if (pot) *pot = phi;
}

/* The field on n particles ((n, 3) arrays; pot may be NULL). */
void oracle_field_all(const oracle_field *f, int64_t n, const double *x,
                      const double *v, double *acc, double *jerk, double *pot) {
  for (int64_t i = 0; i < n; ++i)
    oracle_field_eval(f, &x[3 * i], &v[3 * i], &acc[3 * i], &jerk[3 * i],
                      pot ? &pot[i] : NULL);
}

/* Add the field (if any) to the pair sums of particles idx[0..n_i) whose
 * positions and velocities are x, v. */
static void add_field(const oracle_field *f, int64_t n_i, const int64_t *idx,
                      const double *x, const double *v, double *acc, double *jerk) {
  if (!f) return;
  for (int64_t k = 0; k < n_i; ++k) {
    const int64_t i = idx[k];
    double fa[3], fj[3];
    oracle_field_eval(f, &x[3 * i], &v[3 * i], fa, fj, NULL);
    for (int c = 0; c < 3; ++c) {
      acc[3 * k + c] += fa[c];
      if (jerk) jerk[3 * k + c] += fj[c];
    }
  }
}

/* ---------------------------------------------------------------- energy */

/* Diagnostics of one system (Sect. 4: virial ratio Q = 2K/|W|):
 * out = {K, W, E, Lx, Ly, Lz, Px, Py, Pz} with K = 1/2 sum m v^2,
 * W = -sum_{i<j} m_i m_j / sqrt(r^2 + eps^2), E = K + W + sum_i m_i Phi(x_i)
 * (Phi the external field's potential, none when field is NULL),
 * L = sum m x cross v, P = sum m v.  Pins: Plummer-sphere virial equilibrium
 * (W -> -1/2, K -> 1/4 in Henon units), two-body closed form. */
int oracle_energy(int64_t n, const double *x, const double *v,
                  const double *m, double eps, const oracle_field *field,
                  double *out) {
  if (n < 0 || eps < 0.0) return OR_EINVAL;
  nsum k = {0, 0}, w = {0, 0}, L[3], P[3];
  memset(L, 0, sizeof L);
  memset(P, 0, sizeof P);
  const double eps2 = eps * eps;
  for (int64_t i = 0; i < n; ++i) {
    const double *xi = &x[3 * i], *vi = &v[3 * i];
    nsum_add(&k, 0.5 * m[i] * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]));
    nsum_add(&L[0], m[i] * (xi[1] * vi[2] - xi[2] * vi[1]));
    nsum_add(&L[1], m[i] * (xi[2] * vi[0] - xi[0] * vi[2]));
    nsum_add(&L[2], m[i] * (xi[0] * vi[1] - xi[1] * vi[0]));
    for (int c = 0; c < 3; ++c) nsum_add(&P[c], m[i] * vi[c]);
  }
  int err = OR_OK;
  double *wi = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  if (!wi) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    nsum s = {0, 0};
    for (int64_t j = i + 1; j < n; ++j) {
      const double rx = x[3 * j] - x[3 * i];
      const double ry = x[3 * j + 1] - x[3 * i + 1];
      const double rz = x[3 * j + 2] - x[3 * i + 2];
      const double d2 = rx * rx + ry * ry + rz * rz + eps2;
      if (d2 == 0.0) {
#pragma omp atomic write
        err = OR_EDOMAIN;
        continue;
      }
      nsum_add(&s, -m[i] * m[j] / sqrt(d2));
    }
    wi[i] = nsum_val(&s);
  }
  for (int64_t i = 0; i < n; ++i) nsum_add(&w, wi[i]);
  free(wi);
  nsum we = {0, 0};
  for (int64_t i = 0; field && i < n; ++i) {
    double fa[3], fj[3], phi;
    oracle_field_eval(field, &x[3 * i], &v[3 * i], fa, fj, &phi);
    nsum_add(&we, m[i] * phi);
  }
  out[0] = nsum_val(&k);
  out[1] = nsum_val(&w);
  out[2] = out[0] + out[1] + nsum_val(&we);
  for (int c = 0; c < 3; ++c) {
    out[3 + c] = nsum_val(&L[c]);
    out[6 + c] = nsum_val(&P[c]);
  }
  return err;
}

/* ---------------------------------------------------------------- Hermite */

/* Predictor: Taylor series to the jerk term over dt (Horner form),
 *   xp = x + dt (v + dt (a/2 + dt j/6)),  vp = v + dt (a + dt j/2).
 * Pin: exact for motion with constant jerk (cubic trajectories). */
void oracle_predict_one(const double x[3], const double v[3],
                        const double a[3], const double j[3], double dt,
                        double xp[3], double vp[3]) {
  for (int c = 0; c < 3; ++c) {
    xp[c] = x[c] + dt * (v[c] + dt * (0.5 * a[c] + dt * (j[c] / 6.0)));
    vp[c] = v[c] + dt * (a[c] + dt * (0.5 * j[c]));
  }
}

/* Predict n particles over per-particle intervals dt[i] ((n, 3) arrays). */
void oracle_predict(int64_t n, const double *x, const double *v, const double *a,
                    const double *j, const double *dt, double *xp, double *vp) {
  for (int64_t i = 0; i < n; ++i)
    oracle_predict_one(&x[3 * i], &v[3 * i], &a[3 * i], &j[3 * i], dt[i], &xp[3 * i],
                       &vp[3 * i]);
}

/* Corrector of the fourth-order Hermite scheme over a step h, given the
 * predicted xp, vp and the acceleration and jerk at both ends (a0, j0 at
 * the start, a1, j1 at the end):
 *   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2   (second derivative at start)
 *   a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3     (third derivative)
 *   x1 = xp + a2 h^4/24 + a3 h^5/120,  v1 = vp + a2 h^3/6 + a3 h^4/24
 * and a2_end = a2 + h a3 (second derivative at the end, for the step
 * criterion).  Pin: exact for a cubic-in-time acceleration. */
void oracle_correct_one(const double xp[3], const double vp[3],
                        const double a0[3], const double j0[3],
                        const double a1[3], const double j1[3], double h,
                        double x1[3], double v1[3], double a2_end[3],
                        double a3_out[3]) {
  const double h2 = h * h, h3 = h2 * h;
  for (int c = 0; c < 3; ++c) {
    const double da = a0[c] - a1[c];
    const double a2 = (-6.0 * da - h * (4.0 * j0[c] + 2.0 * j1[c])) / h2;
    const double a3 = (12.0 * da + 6.0 * h * (j0[c] + j1[c])) / h3;
    x1[c] = xp[c] + a2 * (h2 * h2 / 24.0) + a3 * (h2 * h3 / 120.0);
    v1[c] = vp[c] + a2 * (h3 / 6.0) + a3 * (h2 * h2 / 24.0);
    a2_end[c] = a2 + h * a3;
    a3_out[c] = a3;
  }
}

static double norm3(const double a[3]) {
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

/* Aarseth's step criterion
 *   dt = sqrt(eta (|a||a2| + |j|^2) / (|j||a3| + |a2|^2)),
 * +inf when the denominator vanishes. */
double oracle_aarseth_dt(const double a[3], const double j[3],
                         const double a2[3], const double a3[3], double eta) {
  const double na = norm3(a), nj = norm3(j), n2 = norm3(a2), n3 = norm3(a3);
  const double num = na * n2 + nj * nj;
  const double den = nj * n3 + n2 * n2;
  if (den == 0.0) return INFINITY;
  return sqrt(eta * num / den);
}

/* Block-step level update.  Level l means dt = 2^-l.  If the criterion dt_c
 * is below the current step the step is halved until it is <= dt_c (not
 * below 2^-level_max: the clamp is counted in *n_floor).  Otherwise the
 * step is doubled once when dt_c >= 2 dt, the current time t_tick is a
 * multiple of the doubled step, and the doubled step stays <= 2^-level_min.
 * Pins: hand-built commensurability and clamp cases. */
int oracle_next_level(int level, double dt_c, int64_t t_tick, int level_min,
                      int level_max, int64_t *n_floor) {
  double dt = ldexp(1.0, -level);
  if (dt_c < dt) {
    while (dt > dt_c && level < level_max) {
      ++level;
      dt *= 0.5;
    }
    if (dt > dt_c && n_floor) ++*n_floor;
    return level;
  }
  if (level > level_min && dt_c >= 2.0 * dt) {
    const int64_t two_dt_ticks = (int64_t)1 << (OR_TICK_BITS - level + 1);
    if (t_tick % two_dt_ticks == 0) --level;
  }
  return level;
}

/* Initial level: the largest power-of-two step <= eta_s |a| / |j| within
 * [2^-level_max, 2^-level_min] (clamp at the floor counted). */
int oracle_initial_level(const double a[3], const double j[3], double eta_s,
                         int level_min, int level_max, int64_t *n_floor) {
  const double na = norm3(a), nj = norm3(j);
  const double dt0 = (nj == 0.0) ? INFINITY : eta_s * na / nj;
  int level = level_min;
  double dt = ldexp(1.0, -level);
  while (dt > dt0 && level < level_max) {
    ++level;
    dt *= 0.5;
  }
  if (dt > dt0 && n_floor) ++*n_floor;
  return level;
}

/* ---------------------------------------------------------------- driver */

typedef struct {
  double eps, eta, eta_start, dt_shared;
  int32_t level_min, level_max;
  const oracle_field *field;      /* external field, NULL: none */
} oracle_params;

typedef struct {
  int64_t n_block_steps;   /* block steps taken (active-set evaluations) */
  int64_t n_interactions;  /* sum over steps of n_active * n (slots) */
  int64_t n_floor;         /* steps clamped at 2^-level_max */
  int64_t t_tick;          /* time reached, in ticks */
} oracle_stats;

static int finite3(const double a[3]) {
  return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]);
}

/* Initial forces and levels for all n particles at t = 0 (ticks all 0). */
int oracle_init(int64_t n, const double *m, const double *x, const double *v,
                const oracle_params *p, double *a, double *jk,
                int64_t *tick, int8_t *level, oracle_stats *st) {
  if (n <= 0 || !p || p->eps < 0.0 || p->level_min < 0 ||
      p->level_max > OR_MAX_LEVEL || p->level_min > p->level_max)
    return OR_EINVAL;
  int64_t *idx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!idx) return OR_EINVAL;
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  int err = oracle_forces(n, idx, n, x, v, m, p->eps, a, jk, NULL);
  if (!err) add_field(p->field, n, idx, x, v, a, jk);
  free(idx);
  if (err) return err;
  memset(st, 0, sizeof *st);
  st->n_interactions = n * n;
  int shared_level = -1;
  if (p->dt_shared > 0.0) {
    int e;
    double f = frexp(p->dt_shared, &e);   /* dt = 0.5 * 2^e exactly? */
    if (f != 0.5) return OR_EINVAL;
    shared_level = 1 - e;
    if (shared_level < p->level_min || shared_level > p->level_max) return OR_EINVAL;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (!finite3(&a[3 * i]) || !finite3(&jk[3 * i])) return OR_ENONFINITE;
    tick[i] = 0;
    level[i] = (int8_t)(shared_level >= 0
                            ? shared_level
                            : oracle_initial_level(&a[3 * i], &jk[3 * i],
                                                   p->eta_start, p->level_min,
                                                   p->level_max, &st->n_floor));
  }
  return OR_OK;
}

/* Advance the system with Hermite-4 block steps until every particle sits at
 * t_end_tick (which must be a multiple of 2^(20 - level_min) ticks).
 * State arrays are updated in place.  Each block step:
 *   1. T_next = min_i (tick_i + 2^(20 - level_i));
 *      active set A = {i : tick_i + 2^(20 - level_i) == T_next}
 *   2. predict every particle to T_next
 *   3. acceleration and jerk on each i in A from all predicted particles,
 *      plus the external field at i's predicted position and velocity
 *   4. correct each i in A, then choose its next level (block mode) or keep
 *      it (dt_shared > 0)
 * max_steps bounds the number of block steps (0 = no bound). */
int oracle_run(int64_t n, const double *m, double *x, double *v, double *a,
               double *jk, int64_t *tick, int8_t *level,
               const oracle_params *p, int64_t t_end_tick, int64_t max_steps,
               oracle_stats *st) {
  if (n <= 0 || !p) return OR_EINVAL;
  const int64_t dtmax_ticks = (int64_t)1 << (OR_TICK_BITS - p->level_min);
  if (t_end_tick % dtmax_ticks != 0) return OR_EINVAL;
  double *xp = (double *)malloc((size_t)n * 3 * sizeof(double));
  double *vp = (double *)malloc((size_t)n * 3 * sizeof(double));
  double *a1 = (double *)malloc((size_t)n * 3 * sizeof(double));
  double *j1 = (double *)malloc((size_t)n * 3 * sizeof(double));
  int64_t *act = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t steps_here = 0;
  int err = OR_OK;
  if (!xp || !vp || !a1 || !j1 || !act) { err = OR_EINVAL; goto done; }
  const double tick_dt = ldexp(1.0, -OR_TICK_BITS);
  for (int64_t i = 0; i < n; ++i)
    if (tick[i] > st->t_tick) st->t_tick = tick[i];
  for (;;) {
    int64_t t_next = INT64_MAX;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t due = tick[i] + ((int64_t)1 << (OR_TICK_BITS - level[i]));
      if (due < t_next) t_next = due;
    }
    if (t_next > t_end_tick) break;
    if (max_steps > 0 && steps_here >= max_steps) break;
    ++steps_here;
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i)
      if (tick[i] + ((int64_t)1 << (OR_TICK_BITS - level[i])) == t_next) act[na++] = i;
    for (int64_t i = 0; i < n; ++i)
      oracle_predict_one(&x[3 * i], &v[3 * i], &a[3 * i], &jk[3 * i],
                         (double)(t_next - tick[i]) * tick_dt, &xp[3 * i], &vp[3 * i]);
    err = oracle_forces(na, act, n, xp, vp, m, p->eps, a1, j1, NULL);
    if (err) goto done;
    add_field(p->field, na, act, xp, vp, a1, j1);
    for (int64_t k = 0; k < na; ++k) {
      const int64_t i = act[k];
      const double h = (double)(t_next - tick[i]) * tick_dt;
      double a2e[3], a3[3];
      oracle_correct_one(&xp[3 * i], &vp[3 * i], &a[3 * i], &jk[3 * i],
                         &a1[3 * k], &j1[3 * k], h, &x[3 * i], &v[3 * i], a2e, a3);
      for (int c = 0; c < 3; ++c) {
        a[3 * i + c] = a1[3 * k + c];
        jk[3 * i + c] = j1[3 * k + c];
      }
      if (!finite3(&x[3 * i]) || !finite3(&v[3 * i]) || !finite3(&a[3 * i]) ||
          !finite3(&jk[3 * i])) {
        err = OR_ENONFINITE;
        goto done;
      }
      tick[i] = t_next;
      if (p->dt_shared <= 0.0) {
        const double dtc = oracle_aarseth_dt(&a[3 * i], &jk[3 * i], a2e, a3, p->eta);
        level[i] = (int8_t)oracle_next_level(level[i], dtc, t_next, p->level_min,
                                             p->level_max, &st->n_floor);
      }
    }
    st->n_block_steps += 1;
    st->n_interactions += na * n;
    st->t_tick = t_next;
  }
done:
  free(xp);
  free(vp);
  free(a1);
  free(j1);
  free(act);
  return err;
}

/* ------------------------------------------------------ symplectic drivers */

/* Stage weights of the paper's two symplectic schemes (Sect. 4, time
 * integration).  Leapfrog: one stage of weight 1.  Sixth order: the paper
 * takes the first column of Kinoshita, Yoshida & Nakai (1991), Table 1,
 * which is not reproduced in the paper; it is read here as Yoshida's (1990)
 * solution A of the order conditions for a symmetric product of seven
 * second-order leapfrog stages, weights w3 w2 w1 w0 w1 w2 w3 with
 * w0 = 1 - 2 (w1 + w2 + w3).  Returns the number of stages.  Pins: the
 * weights sum to 1, their cubes and fifth powers sum to 0 (the third- and
 * fifth-order error terms of the symmetric product vanish), and the Kepler
 * error falls as h^6. */
int oracle_symplectic_weights(int scheme, double *w) {
  if (scheme == 0) {
    w[0] = 1.0;
    return 1;
  }
  if (scheme != 1) return 0;
  const double w1 = -1.17767998417887;
  const double w2 = 0.235573213359357;
  const double w3 = 0.784513610477560;
  const double w0 = 1.0 - 2.0 * (w1 + w2 + w3);
  const double ws[7] = {w3, w2, w1, w0, w1, w2, w3};
  for (int k = 0; k < 7; ++k) w[k] = ws[k];
  return 7;
}

/* Accelerations of all n particles at positions x (acc-only use of the
 * pair sum above; velocities do not enter the acceleration), plus the
 * external field's. */
static int accel_all(int64_t n, const double *x, const double *m, double eps,
                     const oracle_field *field, double *acc, double *tmp_v,
                     double *tmp_j) {
  int err = OR_OK;
  (void)tmp_v;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double p;
    const double zero[3] = {0.0, 0.0, 0.0};
    int e = force_one(i, &x[3 * i], zero, n, x, tmp_v, m, eps, &acc[3 * i],
                      &tmp_j[3 * i], &p);
    if (e) {
#pragma omp atomic write
      err = e;
    }
    if (field) {
      double fa[3], fj[3];
      oracle_field_eval(field, &x[3 * i], zero, fa, fj, NULL);
      for (int c = 0; c < 3; ++c) acc[3 * i + c] += fa[c];
    }
  }
  return err;
}

/* n_steps steps of size h of the leapfrog (scheme 0) or the sixth-order
 * composition (scheme 1) for one isolated system; x, v ((n, 3)) are updated
 * in place.  Each stage of weight w is the kick-drift-kick leapfrog of step
 * w h: v += (w h / 2) a(x); x += w h v; v += (w h / 2) a(x).  The
 * acceleration at the current positions is kept between stages, so a stage
 * costs one evaluation.  field: external field added to every evaluation
 * (NULL: isolated system).  Pins: Kepler period and convergence order, time
 * reversibility, bounded energy error. */
int oracle_symplectic(int64_t n, const double *m, double *x, double *v,
                      double eps, const oracle_field *field, double h,
                      int64_t n_steps, int scheme) {
  double w[7];
  const int ns = oracle_symplectic_weights(scheme, w);
  if (ns == 0 || n < 1 || n_steps < 0 || !(h > 0.0)) return OR_EINVAL;
  double *a = (double *)calloc((size_t)(3 * n), sizeof(double));
  double *zv = (double *)calloc((size_t)(3 * n), sizeof(double));
  double *jk = (double *)calloc((size_t)(3 * n), sizeof(double));
  int err = (a && zv && jk) ? OR_OK : OR_EINVAL;
  if (!err) err = accel_all(n, x, m, eps, field, a, zv, jk);
  for (int64_t st = 0; st < n_steps && !err; ++st) {
    for (int k = 0; k < ns && !err; ++k) {
      const double c = w[k] * h;
      for (int64_t q = 0; q < 3 * n; ++q) v[q] += 0.5 * c * a[q];
      for (int64_t q = 0; q < 3 * n; ++q) x[q] += c * v[q];
      err = accel_all(n, x, m, eps, field, a, zv, jk);
      for (int64_t q = 0; q < 3 * n; ++q) v[q] += 0.5 * c * a[q];
    }
  }
  free(a);
  free(zv);
  free(jk);
  return err;
}

/* Set the number of OpenMP threads for later calls (no effect without
 * OpenMP); results do not depend on it. */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
