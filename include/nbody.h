/*
 * nbody.h - C ABI of the MI355X direct N-body library (libnbody.so).
 *
 * The library evaluates the O(N^2) pairwise gravitational acceleration of
 * eq. (1) of the paper (Capuzzo-Dolcetta, "Supercomputing and stellar
 * dynamics", Sect. 2), with G = 1 and total mass as the mass unit (Sect. 4),
 * softened in the pair potential by eps (Sect. 4; Plummer form
 * phi = -m / sqrt(r^2 + eps^2)), together with its time derivative (the
 * jerk).  It advances systems with a fourth-order Hermite predictor-corrector
 * on individual power-of-two block time steps chosen by Aarseth's criterion
 * (the paper's individual per-particle time steps, Sect. 3), or with the
 * paper's symplectic drivers (leapfrog and a sixth-order composition,
 * Sect. 4) over an acceleration-only form of the same evaluation.  An
 * optional external Galactic field (Sect. 4; nbody_field) adds to the
 * pairwise forces.  Many independent systems ("clusters") can share one
 * context; each cluster only feels its own particles (and the field).
 *
 * Conventions
 *  - Arrays of vectors are (n, 3) row-major FP64: x[3*i + c].
 *  - All data pointers are DEVICE pointers unless marked "host".
 *  - Time is counted in integer ticks of 2^-20 time units.  A particle on
 *    level l has step 2^-l; levels run from level_min (largest step) to
 *    level_max (smallest step), 0 <= level_min <= level_max <= 20.
 *  - Calls are asynchronous on params.stream unless marked "syncs".
 *  - Return values are NBODY_OK (0) or a negative nbody_status.  Arguments
 *    that can be checked on the host are checked before any device work.
 *    Errors found by kernels are sticky: they are returned by the next call
 *    that syncs (nbody_step, nbody_energy, nbody_get_state, nbody_sync).
 *  - No exceptions cross this interface.  nbody_last_error() gives a
 *    human-readable message for the calling thread's last failure.
 *
 * Ownership
 *  - The caller owns every buffer passed in, including the device workspace
 *    and the stream.  The library never allocates or frees device memory; it
 *    carves its state out of the workspace.  A context must be destroyed
 *    before its workspace is freed or reused.
 *  - nbody_init copies the initial state into the workspace; the caller's
 *    m, x, v may be freed afterwards.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nbody_ctx nbody_ctx;

typedef enum nbody_status {
  NBODY_OK = 0,
  NBODY_EINVAL = -1,     /* invalid argument (host-checked, nothing enqueued) */
  NBODY_ENODEV = -2,     /* no usable HIP device */
  NBODY_ENOMEM = -3,     /* workspace smaller than nbody_workspace_bytes() */
  NBODY_EHIP = -4,       /* a HIP runtime call failed */
  NBODY_EINDEX = -5,     /* device-detected: an i index out of range or
                            i_active not grouped by cluster */
  NBODY_ENONFINITE = -6, /* device-detected: NaN/Inf in forces or state */
  NBODY_EDOMAIN = -7     /* device-detected: eps == 0 and two distinct
                            particles at the same position */
} nbody_status;

typedef enum nbody_precision {
  /* plain FP64 arithmetic throughout */
  NBODY_FP64 = 0,
  /* FP64 state, predictor and corrector; x_j - x_i is an FP64 subtraction
     of the FP64 predicted positions rounded to FP32; v_j - v_i is
     (v_j - v_ref) rounded to FP32 minus the i-particle's v_i - v_ref held
     as an exact (hi, lo) FP32 pair, v_ref being each cluster's reference
     velocity (the mass-weighted mean velocity of a strided sample of up to
     256 of its particles), so it carries only the rounding of v_j - v_ref;
     then FP32 r^2, r.v, rsqrt, r^-3 and jerk products (the hardware
     rsqrt corrected by its FMA residual); FP32 sums of every 64 j folded
     into a compensated (TwoSum) FP32 hi/lo pair.  Pairs that dominate a
     particle's jerk are evaluated in FP64 instead (near pairs, see
     nbody_tuning.near_jerk), and particles whose acceleration is dominated
     by a single term (nbody_tuning.refine_ratio) are re-evaluated in FP64;
     acceleration and jerk then meet 1e-6 relative. */
  NBODY_MIXED = 1,
  /* as NBODY_MIXED, but x_j - x_i and v_j - v_i formed in FP32 from the
     FP64 predicted positions and velocities split into double-single pairs
     (the paper's software double precision, Sect. 5): (hi_j - hi_i) +
     (lo_j - lo_i), within an FP32 ulp of the FP64 difference (j records of
     64 bytes) */
  NBODY_MIXED_DS = 2
} nbody_precision;

/* External Galactic field added to the pairwise forces (Sect. 4: the paper
 * sums the star-star forces with an analytic Galactic potential, the model
 * of Allen & Santillan (1991) with a spherical bulge, an axisymmetric disk
 * and a spherical halo; the paper gives neither formulas nor parameters).
 * Positions are taken about the Galactic centre, z along the disk axis;
 * every value in the context's units with G = 1:
 *   bulge  Phi = -bulge_m / sqrt(r^2 + bulge_b^2)                (Plummer)
 *   disk   Phi = -disk_m / sqrt(R^2 + (disk_a + sqrt(z^2 + disk_b^2))^2)
 *                                                     (Miyamoto & Nagai)
 *   halo   enclosed mass M(r) = halo_m s^(g + 1) / (1 + s^g), s = r / halo_a,
 *          g = halo_gamma, up to r = halo_rc and M(halo_rc) beyond; radial
 *          pull M(r) / r^2 and the potential that integrates it from
 *          infinity (no pull at r = 0).
 * A zero mass switches a component off; the other values of an active
 * component must be finite, lengths > 0 (disk_a >= 0), halo_gamma > 0.
 * Allen & Santillan's model in units of 1 kpc and 2.32e7 M_sun: bulge
 * 606, 0.3873; disk 3690, 5.3178, 0.25; halo 4615, 12, 1.02, 100. */
typedef struct nbody_field {
  double bulge_m, bulge_b;
  double disk_m, disk_a, disk_b;
  double halo_m, halo_a, halo_gamma, halo_rc;
} nbody_field;

typedef struct nbody_params {
  int32_t n_clusters;              /* >= 1, <= 4096 */
  int32_t precision;               /* nbody_precision */
  const int64_t *cluster_offsets;  /* host, n_clusters + 1 entries, [0] = 0,
                                      strictly increasing, last = n; NULL
                                      means one cluster [0, n) */
  const double *eps;               /* host, n_clusters softening lengths >= 0 */
  double eta;                      /* Aarseth accuracy parameter, > 0 */
  double eta_start;                /* initial step: eta_start |a| / |jerk|, > 0 */
  double dt_shared;                /* > 0: every particle uses this step
                                      (a power of two in [2^-level_max,
                                      2^-level_min]); 0: block steps */
  int32_t level_min, level_max;    /* step range [2^-level_max, 2^-level_min] */
  void *stream;                    /* hipStream_t for all work; NULL = null stream */
  void *workspace;                 /* device buffer, 256-byte aligned */
  size_t workspace_bytes;          /* >= nbody_workspace_bytes(params, n) */
  const nbody_field *field;        /* host, read at nbody_init; NULL: no
                                      external field.  When set, its
                                      acceleration and jerk are added to the
                                      pairwise ones wherever the integrators
                                      use them (the stored a and jerk, block
                                      and symplectic steps) and its potential
                                      energy to E; nbody_forces and
                                      nbody_accel stay pairwise. */
} nbody_params;

/* Bytes of device workspace a context for n particles needs (0 if the
 * parameters are invalid).  Host only; no device call. */
size_t nbody_workspace_bytes(const nbody_params *p, int64_t n);

/* Create a context for n particles, copy masses m (n), positions x and
 * velocities v ((n, 3), device) into the workspace, evaluate the initial
 * acceleration (Sect. 2, eq. (1), softened as in Sect. 4) and its time
 * derivative, the jerk, of every particle, and choose initial levels of the
 * individual block time steps (Sect. 3)
 * (dt_shared, or the largest power-of-two step <= eta_start |a| / |jerk|,
 * clamped to the level range).  All particles start at t = 0.  Syncs.
 * *out is set to NULL on failure. */
int nbody_init(nbody_ctx **out, const nbody_params *p, int64_t n,
               const double *m, const double *x, const double *v);

/* Pure evaluation (eq. (1) with Plummer softening, plus jerk): for k in
 * [0, n_active), acc[k] and jerk[k] ((n_active, 3), device) receive the sum
 * over the j-particles xj, vj ((n_j, 3)) and mj (n_j) of the pair terms on
 * particle i = i_active[k] (an index into the j arrays), skipping j == i.
 * With one cluster n_j may be any size >= 1; with several clusters n_j must
 * equal the context's n, i's partners are the particles of its own cluster,
 * and i_active must be grouped by cluster (non-decreasing cluster id).
 * Indices may repeat.  The context's state is not touched; its precision,
 * softening and stream are used.  Asynchronous; an index out of range or a
 * grouping violation is reported as NBODY_EINDEX at the next syncing call
 * and the affected outputs are zero. */
int nbody_forces(nbody_ctx *c, const int32_t *i_active, int64_t n_active,
                 const double *xj, const double *vj, const double *mj,
                 int64_t n_j, double *acc, double *jerk);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the evaluation of
 * nbody_forces for one cluster without a context, allocating nothing.
 * acc[k] and jerk[k] ((n_active, 3), device; jerk may be NULL) receive the
 * pair sums over xj, vj ((n_j, 3), device) and mj (n_j, device) on particle
 * i_active[k] (device), skipping j == i, with softening eps >= 0, in the
 * given precision (nbody_precision, default tuning), enqueued on stream
 * (hipStream_t; NULL = null stream) and asynchronous.  Limits: n_j in
 * [1, 16384] and n_active <= 16384 (NBODY_EINVAL otherwise).  Its scratch
 * is a fixed 16 MiB device array in the library, one per GPU, held until the
 * process ends; calls that overlap on one GPU (other streams, other host
 * threads' streams) race on it and must be ordered by the caller.  An index
 * out of range leaves that entry's outputs zero; no error is reported for
 * it (there is no context to hold a sticky error). */
int nbody_forces_noalloc(int precision, double eps, const int32_t *i_active,
                         int64_t n_active, const double *xj, const double *vj,
                         const double *mj, int64_t n_j, double *acc, double *jerk,
                         void *stream);

/* Acceleration only (eq. (1) with Plummer softening; the force function of
 * the paper's symplectic drivers): acc[k] ((n_active, 3), device) receives
 * the sum over xj ((n_j, 3)) and mj (n_j) of the pair accelerations on
 * i = i_active[k], skipping j == i.  Same rules as nbody_forces for n_j,
 * clusters, grouping, repeats, errors and asynchrony; no velocities are
 * read.  The mixed path's FP64 re-evaluation applies as in nbody_forces. */
int nbody_accel(nbody_ctx *c, const int32_t *i_active, int64_t n_active,
                const double *xj, const double *mj, int64_t n_j, double *acc);

/* The paper's symplectic drivers (Sect. 4, time integration):
 * NBODY_LEAPFROG, the second-order kick-drift-kick leapfrog (one force
 * evaluation per step), and NBODY_SYMPLECTIC6, the sixth-order explicit
 * scheme built as the symmetric composition of seven leapfrog stages with
 * Yoshida's solution A weights (seven evaluations per step). */
enum { NBODY_LEAPFROG = 0, NBODY_SYMPLECTIC6 = 1 };

/* Advance every particle by n_steps steps of the constant size h with a
 * symplectic driver, using acceleration-only evaluations in the context's
 * precision (consecutive half kicks merge, so a step costs one evaluation
 * per stage, plus one at the start of the call since the state's
 * accelerations were taken at predicted positions).  Every particle must
 * sit at its cluster's time (true after nbody_init and nbody_step;
 * otherwise NBODY_EINVAL at the end of the call).  h must be a positive
 * multiple of 2^-20 and n_steps * h a multiple of 2^-level_min, so that
 * block steps can follow.  On return every time has advanced by
 * n_steps * h and acceleration, jerk and levels are re-evaluated at the new
 * positions, as nbody_init does.  n_interactions (if non-NULL) receives
 * the pair slots of the acceleration evaluations.  Syncs. */
int nbody_step_symplectic(nbody_ctx *c, int scheme, double h, int64_t n_steps,
                          int64_t *n_interactions);

/* Advance every cluster with Hermite-4 block steps (the individual,
 * per-particle time steps of Sect. 3, over the force of Sect. 2 eq. (1)
 * with the softening of Sect. 4) to the absolute time
 * t_end, which must be a multiple of 2^-level_min and not earlier than the
 * current time.  Each block step: per cluster, the next time
 * T_next = min_i (t_i + dt_i) and the active set {i : t_i + dt_i = T_next};
 * every particle of the cluster predicted to T_next; acceleration and jerk
 * of the active particles; correction; new levels.  Steps run as captured
 * HIP graphs unless tuning says otherwise.  If n_block_steps is non-NULL it
 * receives the number of device block-step iterations taken by this call;
 * n_interactions the sum of n_active * n_cluster over them.  Syncs. */
int nbody_step(nbody_ctx *c, double t_end, int64_t *n_block_steps,
               int64_t *n_interactions);

/* As nbody_step, but stop after at most max_block_steps block-step
 * iterations (eager launches, no graph): for output or checks at block-step
 * granularity.  Clusters may stop short of t_end, each at the time of its
 * last block step, with particles in the middle of their own steps; a later
 * nbody_step or nbody_step_blocks continues from there.  Syncs. */
int nbody_step_blocks(nbody_ctx *c, double t_end, int64_t max_block_steps,
                      int64_t *n_block_steps, int64_t *n_interactions);

/* Diagnostics per cluster, computed in FP64 at each cluster's current time
 * (every particle predicted to it): out (host) receives 9 doubles per
 * cluster: K, W, E, Lx, Ly, Lz, Px, Py, Pz, with K = 1/2 sum m v^2,
 * W = -sum_{i<j} m_i m_j / sqrt(r^2 + eps^2), E = K + W (+ sum m Phi_ext(x)
 * with an external field), L = sum m x cross v, P = sum m v (virial ratio
 * Q = 2K/|W|, Sect. 4).  Syncs. */
int nbody_energy(nbody_ctx *c, double *out);

/* Copy the state out: x, v, a, jerk ((n, 3), device, FP64), tick (n, int64,
 * device: time of each particle's last correction in ticks), level (n,
 * int8, device).  Any pointer may be NULL to skip it.  Syncs. */
int nbody_get_state(nbody_ctx *c, double *x, double *v, double *a,
                    double *jerk, int64_t *tick, int8_t *level);

/* Replace the state (same layouts as nbody_get_state, none may be NULL).
 * Each cluster's current time becomes the largest tick among its
 * particles.  Every particle must satisfy: level in the level range, tick a
 * multiple of its step 2^(20 - level), tick <= cluster time < tick + step
 * (otherwise NBODY_EINVAL).  Syncs. */
int nbody_set_state(nbody_ctx *c, const double *x, const double *v,
                    const double *a, const double *jerk, const int64_t *tick,
                    const int8_t *level);

/* Wait for the context's stream and return the sticky device error, if any
 * (the error is cleared once returned). */
int nbody_sync(nbody_ctx *c);

/* Per-context counters since nbody_init (host, 8 int64): block steps,
 * interactions (n_active * n_cluster summed over steps), clamps at the
 * smallest step, current time of cluster 0 in ticks, particles re-evaluated
 * in FP64 by the mixed path (steps and nbody_forces), near pairs evaluated
 * in FP64 by the mixed path (see nbody_tuning.near_jerk), interactions of
 * mixed block steps that ran on the FP64 kernel (steps with few active
 * particles), and 1 reserved.  Syncs. */
int nbody_stats(nbody_ctx *c, int64_t *out8);

/* Kernel timing for measurement.  While enabled, block steps launch their
 * kernels eagerly (no graph; results are identical) and the library records
 * a pair of HIP events on the context's stream around every launch of the
 * force kernel (steps and nbody_forces).  nbody_profile_read syncs and
 * returns, since the previous read, the summed event time in ms and the
 * number of launches of the context's own force kernel (FP64 or mixed) and,
 * separately, of the FP64 re-evaluation launches of the mixed path (any
 * pointer may be NULL). */
int nbody_profile(nbody_ctx *c, int enable);
int nbody_profile_read(nbody_ctx *c, double *force_ms, int64_t *force_launches,
                       double *refine_ms, int64_t *refine_launches);

/* Free the host-side context (the workspace stays with the caller).  Waits
 * for outstanding work.  NULL is ignored. */
void nbody_destroy(nbody_ctx *c);

const char *nbody_strerror(int code);
const char *nbody_last_error(void);

/* ---- launch tuning (written by the autotuner, optional) ----------------
 * The force kernel runs over work items (cluster, i-tile, j-split).  For a
 * cluster with n_active particles in bucket b = floor(log2(n_active))
 * (0..24), i_slots[b] threads of a 256-thread workgroup hold i-particles
 * (a power of two, 1..256; the other 256 / i_slots lanes split j inside the
 * workgroup) and the j range is split until the cluster has about
 * target_items[b] items (1..2^20), within two bounds: no split shorter than
 * min_split_j, and splits x n_active <= 32 n_j (the partial-sum rows the
 * workspace holds per j-particle).  variant selects the compiled kernel shape:
 * NBODY_VARIANT_K1 (one i per thread slot) or NBODY_VARIANT_K2 (two), both
 * staging j through LDS; NBODY_VARIANT_S1 / _S2 add the broadcast kernel
 * (j records read into scalar registers) for evaluations with at least
 * n_j / 16 active particles and i_slots = 256 in every cluster, with one or
 * two i per lane (the LDS kernel with the same K takes the others).  All
 * variants with the same K give bitwise-identical results.
 * Zero fields keep the defaults. */
#define NBODY_TUNE_BUCKETS 25
enum { NBODY_VARIANT_DEFAULT = 0, NBODY_VARIANT_K1 = 1, NBODY_VARIANT_K2 = 2,
       NBODY_VARIANT_S1 = 3, NBODY_VARIANT_S2 = 4 };
enum { NBODY_GRAPH_ON = 1, NBODY_GRAPH_OFF = 2 };

typedef struct nbody_tuning {
  int32_t variant;
  int32_t use_graph;        /* NBODY_GRAPH_ON: block steps replay a captured
                               HIP graph (default); NBODY_GRAPH_OFF: eager
                               launches (results are identical) */
  int32_t steps_per_launch; /* block steps per graph launch / host check */
  int32_t min_split_j;      /* smallest j range of one split (>= 64) */
  float refine_ratio;       /* mixed path: particles whose largest single
                               acceleration term, bounded by max_j m_j/s_ij,
                               exceeds refine_ratio times their net
                               acceleration are re-evaluated with the FP64
                               kernel (default 1; < 0 disables) */
  int32_t i_slots[NBODY_TUNE_BUCKETS];
  int32_t target_items[NBODY_TUNE_BUCKETS];
  int32_t acc_variant;      /* variant of the acceleration-only evaluations
                               (nbody_accel, the symplectic drivers), whose
                               lighter kernels may prefer another one;
                               0: the same as variant.  In nbody_set_tuning
                               0 keeps the current value and -1 resets it
                               to 0. */
  float near_jerk;          /* mixed paths, evaluations with jerk: a pair
                               whose jerk scale m_j s_ij^-3/2 max_c
                               |v_j,c - v_i,c| exceeds near_jerk times an
                               estimate of i's jerk is evaluated in FP64 and
                               left out of the FP32 sums (the few close
                               neighbours whose terms set the FP32 error of
                               the jerk; 3-6 pairs per particle at the
                               default 0.0625).  The estimate is a first
                               FP64-free pass over the same evaluation
                               (nbody_init, nbody_forces, the closing
                               evaluation of nbody_step_symplectic), and a
                               particle whose estimate exceeds twice its
                               jerk is re-evaluated in FP64; in block steps
                               it is the particle's stored jerk, with the
                               threshold halved and four times its jerk as
                               the bound.  < 0 turns near pairs off. */
  int32_t small_log2;       /* mixed paths, block steps: a cluster whose step
                               has at most 256 active particles or at most
                               2^small_log2 interactions (n_active x N_c) is
                               evaluated by the FP64 kernel, which predicts
                               its j-particles on the fly and needs neither
                               j records nor near pairs (default 27).  In
                               nbody_set_tuning 0 keeps the current value
                               and -1 routes every block step through the
                               mixed kernels; otherwise 1..62.  nbody_stats
                               counts the interactions so routed. */
} nbody_tuning;

/* Read or replace the tuning of a context (host only, no device work). */
int nbody_get_tuning(const nbody_ctx *c, nbody_tuning *t);
int nbody_set_tuning(nbody_ctx *c, const nbody_tuning *t);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
