// Internal types shared by the host runtime (nbody_api.cpp) and the device
// kernels (nbody_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace nbk {

constexpr int kWG = 256;            // threads per workgroup of every kernel
constexpr int kTJ = 256;            // j records per LDS tile of the force kernel
constexpr int kTickBits = 20;       // one time unit = 2^20 ticks
constexpr int kLevels = 21;         // levels 0..20, step 2^-level
constexpr int kMaxClusters = 4096;
constexpr int kScanBlock = 1024;    // particles per block of the compaction
constexpr int kFusedScan = 1024;    // compaction grids up to this many blocks
                                    // (N <= 2^20) skip the separate scan
constexpr int kBuckets = 25;        // tuning buckets floor(log2(n_active))
constexpr int kNoActive = 99;       // threshold level meaning "nothing due"
constexpr int kSmallStep = 256;     // mixed block steps up to this many active
                                    // particles are evaluated by the FP64 kernel,
                                    // and so are those of up to Tuning::small_work
                                    // interactions (n_active x N_c)
constexpr int kRowsPerJ = 32;       // partial rows a cluster may take per j-particle
constexpr int kRowStride = 8;       // doubles per partial row: a(3), jerk(3),
                                    // bound on the largest acc term, far-field
                                    // jerk scale (double-single)
constexpr double kFarRatio = 8.0;   // double-single: a far-field jerk scale
                                    // above this many times the jerk sends the
                                    // particle to FP64
constexpr double kNearStale = 2.0;  // a near-pair threshold taken from a jerk
                                    // estimate more than this many times the
                                    // jerk found sends the particle to FP64
constexpr double kNearStaleState = 4.0;   // the same for block steps, whose
                                    // thresholds are halved (stored jerk)

// kErrState: a state given to nbody_set_state, or found by a driver, that
// breaks the block-step invariants
enum ErrBits : int32_t { kErrNonFinite = 1, kErrDomain = 2, kErrIndex = 4, kErrState = 8 };

// counters in Dev::ctr
enum Ctr : int {
  kCtrSteps = 0,        // block-step iterations with work
  kCtrInter = 1,        // sum of n_active * n_cluster
  kCtrFloor = 2,        // steps clamped at 2^-level_max
  kCtrNotDone = 3,      // clusters still short of t_end after the last step
  kCtrTend = 4,         // t_end in ticks for nbody_step
  kCtrRefined = 5,      // entries re-evaluated in FP64 (mixed path)
  kCtrNear = 6,         // near pairs evaluated in FP64 (mixed path)
  kCtrSmallInter = 7,   // interactions of mixed block steps run by the FP64
                        // kernel (small steps)
  kCtrCount = 8
};

// Per-cluster launch plan of one force evaluation.  Built on the device by
// k_plan so that a captured graph adapts to the active-set sizes.
struct ClusterPlan {
  int32_t c;        // cluster id
  int32_t P;        // i thread-slots per workgroup (power of two, 1..256)
  int32_t Qlog;     // log2 of j-lanes per i slot (Q = 256 / P)
  int32_t S;        // j splits
  int32_t na;       // active particles of the cluster
  int32_t act_off;  // their offset in the active list
  int32_t tiles;    // i tiles = ceil(na / (P * K))
  int32_t items;    // tiles * S
  int64_t row_off;  // first partial row of the cluster
  int64_t jb, je;   // j range [jb, je)
  int64_t chunk;    // j per split (multiple of kTJ)
  int64_t t_pred;   // tick every particle of the cluster is predicted to
  int32_t small;    // small mixed block step (kSmallStep, Tuning::small_work):
                    // evaluated by the FP64 kernel, never re-evaluated
  int32_t glog;     // log2 of the lanes that sum one entry's S rows
                    // (the power of two >= S, at most 64)
};

struct Tuning {     // device copy of the launch policy (passed by value)
  int32_t i_slots[kBuckets];
  int32_t target_items[kBuckets];
  int32_t min_split_j;
  int32_t K;        // i-particles per thread slot (1 or 2)
  int64_t small_work;   // small mixed block steps: at most this many
                        // interactions, or kSmallStep active; < 0: none
};

// Plan kinds (k_plan): which time the particles are predicted to, where the
// j range comes from, and whether the step is committed.
enum PlanKind : int {
  kPlanStep = 0,     // block step: predict to T_next, commit T = T_next, count
  kPlanState = 1,    // init / energy: predict to T
  kPlanApi = 2,      // nbody_forces: caller's j arrays
  kPlanRefine = 3,   // FP64 re-evaluation inside a block step (T_next)
  kPlanApiRefine = 4 // FP64 re-evaluation inside nbody_forces
};

// Device pointers carved from the caller's workspace.
// External field (see nbody_field), with the halo constants the host
// derives: mass inside the cut-off and the potential's inner offset.
struct Field {
  double bm, bb;             // bulge mass, scale
  double dm, da, db;         // disk mass, radial and vertical scales
  double hm, ha, hg, hrc;    // halo mass scale, radius, exponent, cut-off
  double hmc;                // M(hrc)
  double hpc;                // inner potential: hpc + hm / (hg ha) ln(1 + s^hg)
  int32_t on, pad_;
};

struct Dev {
  int64_t n;
  int32_t C;
  int32_t nblk;        // compaction blocks = ceil(n / kScanBlock)
  int64_t rows_cap;    // partial rows available
  int64_t cap_active;  // entries of the active list
  // particle state, component-major SoA: x[c * n + i]
  double *x, *v, *a, *j;
  double *m;
  int64_t *tick;
  int32_t *level;
  int32_t *cid;
  // clusters
  int64_t *coff;       // C + 1
  double *eps2;        // C
  int64_t *T;          // C: current time
  int64_t *Tnext;      // C: time of the block step being taken
  int32_t *Lthr;       // C: levels >= Lthr are due at Tnext
  int32_t *hist;       // C * kLevels: particles per level
  // active list and compaction
  int32_t *active;     // cap_active
  int32_t *act_off;    // C + 1
  int32_t *blk_cnt;    // nblk: due particles per compaction block
  int32_t *flag_cnt;   // nblk: flagged entries per block of the active list
  int32_t *blk_off;    // nblk + 1
  // plan
  ClusterPlan *plan_c;    // C, by cluster id
  ClusterPlan *plan_lpt;  // C, largest item cost first
  int32_t *item_prefix;   // C + 1 (LPT order)
  int32_t *sum_prefix;    // C + 1 (cluster order): waves of the row sums
  double *partial;        // rows_cap * kRowStride
  // per active entry k: summed acceleration and jerk, refinement flag
  double *fsum;           // cap_active * 6
  int32_t *rflag;         // cap_active
  int32_t *ref_i;         // cap_active: particles re-evaluated in FP64
  int32_t *ref_k;         // cap_active: their active-list positions
  int32_t *ref_off;       // C + 1: per-cluster offsets in ref_i (last = count)
  float *theta;           // cap_active: near-pair threshold of each entry,
                          // from the first pass of a two-pass evaluation
  // j records of an evaluation with many active particles
  void *pred;             // n records of 64 bytes (the LDS record format)
  int32_t *pred_on;       // 0 none, 1 built, 2 built for the broadcast kernel
  // words
  int32_t *work;       // [0] main item counter, [1] small-step item counter,
                       // [2] number of main items (written by k_plan)
  double *vref;        // 3 * C: each cluster's reference velocity of the
                       // FP64-difference mixed records (k_vref)
  int32_t *sync;       // [0] flagged-entry count, [1] finished blocks of an
                       // appending k_sum_flag (both zero between launches)
  int32_t *err;        // sticky error bits
  int64_t *ctr;        // kCtrCount counters
  double *eout;        // C * 9 energy output
  Field fld;           // external field (fld.on == 0: none)
};

// Where the force kernel takes j (and i) particles from: the state
// (predicted while the tile is filled, or the records when built), the
// caller's arrays, or only the records (launches that always have them).
enum Source : int { kSrcState = 0, kSrcRaw = 1, kSrcRec = 2 };
// What the force kernel computes: acceleration and jerk, the potential, or
// the acceleration alone (the symplectic drivers and nbody_accel); in FP64,
// mixed with double-single differences, or mixed with FP64 differences.
enum Mode : int {
  kModeFP64 = 0,
  kModeMixed = 1,
  kModePot = 2,
  kModeFP64Acc = 3,
  kModeMixedAcc = 4,
  kModeMixed64 = 5,
  kModeMixed64Acc = 6
};
constexpr bool mode_acc_only(int m) {
  return m == kModeFP64Acc || m == kModeMixedAcc || m == kModeMixed64Acc;
}
// FP32 pair arithmetic: compensated FP32 sums, the largest-term bound and
// the FP64 re-evaluation
constexpr bool mode_mixed(int m) {
  return m == kModeMixed || m == kModeMixedAcc || m == kModeMixed64 || m == kModeMixed64Acc;
}

// Near pairs of the mixed evaluations with jerk (evaluated in FP64, left out
// of the FP32 sums): the threshold of each i is c times a jerk estimate,
// the magnitude of its stored jerk (kNearState: block steps) or the first
// pass's jerk of its entry (kNearList: d.theta holds c |jerk| already);
// kNearNone: no near pairs.
enum NearSrc : int { kNearNone = 0, kNearState = 1, kNearList = 2 };
struct NearSpec {
  int src;
  float c;
};
// Host-side launchers (defined in nbody_kernels.hip).  Every launcher only
// enqueues on `s`; none synchronises.  They return the hipError_t of the
// launch.
struct RawSrc {                 // caller arrays for nbody_forces
  const double *x, *v, *m;     // (n_j, 3), (n_j, 3), (n_j)
  int64_t n_j;                 // j count (single cluster) or 0 (use coff)
  const int32_t *i_active;     // n_active indices
  int64_t n_active;
  double *acc, *jerk;          // (n_active, 3) outputs
};

hipError_t launch_init_state(const Dev &d, const double *m, const double *x,
                             const double *v, hipStream_t s);
// Every particle active; with one cluster also the kPlanState plan (tuning t).
hipError_t launch_all_active(const Dev &d, const Tuning &t, hipStream_t s);
// One-cluster contexts whose compaction takes its block prefixes itself:
// the compaction kernels also write the plan that follows (launch_compact
// the block step's, launch_sum_and_flag the re-evaluation's), and the
// separate launch_plan is skipped.
bool plan_fused(const Dev &d);
// Scheduler (per-cluster T_next and threshold level) and ordered compaction
// of the due particles into the active list (plan: see plan_fused).
// rec_mode >= 0 (a force mode; one cluster with plan_fused): the compaction
// also writes every particle's j record predicted to T_next and the record
// flag (allow_sb, sb_only as in launch_records), so no launch_records
// follows; -1: records are left to launch_records.
hipError_t launch_compact(const Dev &d, const Tuning &t, bool allow_small, int rec_mode,
                          bool allow_sb, bool sb_only, hipStream_t s);
// allow_small: clusters of a small block step (at most kSmallStep active
// particles, or at most Tuning::small_work interactions) are planned for the
// small-step FP64 launch (mixed contexts).  A re-evaluation plan also
// writes the per-cluster offsets of the re-evaluation list (ref_off).
hipError_t launch_plan(const Dev &d, const Tuning &t, int kind,
                       int64_t api_nj, bool allow_small, hipStream_t s);
// Hermite corrector parameters of a block step.
struct CorrectSpec {
  double eta, dt_shared;
  int lmin, lmax;
};
// Sum each active entry's partial rows into fsum.  theta_out (first pass of
// a two-pass mixed evaluation): store each entry's near-pair threshold
// nr.c |jerk| in d.theta.  Otherwise, with refine_ratio > 0, flag the entries
// whose largest acceleration term exceeds refine_ratio times their net
// acceleration or whose near-pair threshold came from a jerk estimate above
// kNearStale times their jerk (nr.src), and build the grouped re-evaluation
// list.
// append (block steps): with one cluster and a fused plan, the flagged
// entries are appended to the list in any order and the sum launch writes
// the re-evaluation plan (no k_rscatter).
hipError_t launch_sum_and_flag(const Dev &d, const int32_t *list, int64_t na_host,
                               float refine_ratio, const NearSpec &nr, bool theta_out,
                               const Tuning &t1, int ref_kind, int64_t api_nj, bool append,
                               hipStream_t s);
// Overwrite fsum of the re-evaluated entries with their FP64 sums; corr
// (block steps): and apply the corrector to every active particle, so no
// launch_correct follows.
hipError_t launch_refine_finalize(const Dev &d, const CorrectSpec *corr, hipStream_t s);
// Which work a force launch takes.  The plan splits the items in two:
// [0, work[2]) for the main launches, [work[2], total) for the small-step
// launch.  kRoleAlways: the main items, whatever the record flag
// (re-evaluation, potential); kRoleMain: the main items unless the record
// flag (*d.pred_on, set by launch_records) is 2 — then the broadcast kernel
// takes them — reading records when it is 1; kRoleSmall: the small-step
// items (clusters of a small mixed block step), in FP64 with the prediction
// fused into the tile fill.
enum Role : int { kRoleAlways = 0, kRoleMain = 1, kRoleSmall = 2 };
hipError_t launch_force(const Dev &d, int mode, int src, int K,
                        const RawSrc *raw, const int32_t *list, int role,
                        const NearSpec &nr, int grid, hipStream_t s);
// Build the records of one evaluation into d.pred when its active set is at
// least 1/16 of its j particles, and set *d.pred_on (0, 1, or 2 when the
// broadcast kernel may take it: allow_sb and kWG i-slots in every cluster
// with work for the main kernels).
// kind: kPlanStep (predict to T_next), kPlanState (to T), kPlanApi (raw).
// sb_only: the caller enqueues no workgroup-kernel launch for the main items,
// so a record flag other than 2 is reported as kErrState.
hipError_t launch_records(const Dev &d, int mode, int kind, const RawSrc *raw,
                          bool allow_sb, bool always, bool sb_only, hipStream_t s);
// The broadcast force kernel (j records in scalar registers); it does the
// evaluation only when *d.pred_on == 2 and returns at once otherwise.
hipError_t launch_force_sb(const Dev &d, int mode, int K, const RawSrc *raw,
                           const int32_t *list, const NearSpec &nr, int grid, hipStream_t s);
int force_sb_grid_size(int mode, int K, int device);
// Symplectic drivers: kick (v += ck a, a from fsum) then drift (x += cd v)
// (with one cluster also the next evaluation's kPlanState plan, tuning t);
// final kick; advance all times by dticks.
hipError_t launch_sym_kick_drift(const Dev &d, double ck, double cd, bool check,
                                 const Tuning &t, hipStream_t s);
hipError_t launch_sym_kick(const Dev &d, double ck, hipStream_t s);
hipError_t launch_sym_advance(const Dev &d, int64_t dticks, hipStream_t s);
// Each cluster's reference velocity for the FP64-difference mixed records
// (the mass-weighted mean velocity of a strided sample of the cluster), from
// the state, or from a caller's arrays (raw, which must carry velocities).
hipError_t launch_vref(const Dev &d, const RawSrc *raw, hipStream_t s);
// Row sums of the step plan's partial rows and the corrector in one launch
// (block steps without a re-evaluation pass; with one, the re-evaluation's
// launch_refine_finalize corrects).
hipError_t launch_correct(const Dev &d, double eta, double dt_shared,
                          int level_min, int level_max, hipStream_t s);
hipError_t launch_init_levels(const Dev &d, double eta_start,
                              double dt_shared, int level_min, int level_max,
                              hipStream_t s);
// nbody_forces / nbody_accel: per-cluster offsets of the caller's active list
// (and its index checks); with one cluster also the kPlanApi plan (tuning t).
hipError_t launch_api_group(const Dev &d, const RawSrc &r, const Tuning &t, hipStream_t s);
hipError_t launch_api_finalize(const Dev &d, const RawSrc &r, hipStream_t s);
hipError_t launch_energy_reduce(const Dev &d, hipStream_t s);
hipError_t launch_set_word64(int64_t *p, int64_t v, hipStream_t s);
hipError_t launch_fill32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_get_state(const Dev &d, double *x, double *v, double *a,
                            double *jk, int64_t *tick, int8_t *level,
                            hipStream_t s);
hipError_t launch_set_state(const Dev &d, const double *x, const double *v,
                            const double *a, const double *jk,
                            const int64_t *tick, const int8_t *level,
                            int level_min, int level_max, hipStream_t s);
// persistent grid size of the force kernel (workgroups resident at once)
int force_grid_size(int mode, int src, int K, int device);

}  // namespace nbk
