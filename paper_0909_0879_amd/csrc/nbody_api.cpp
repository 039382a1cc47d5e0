// Host runtime of libnbody.so: argument validation, workspace carving,
// launch sequencing and HIP-graph capture of block steps.  See nbody.h for
// the contract of every entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nbody.h"
#include "nbody_internal.h"

using nbk::Dev;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define NB_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(NBODY_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kEvPairs = 1024;
// mixed path: re-evaluate in FP64 the particles whose largest acceleration
// term exceeds this multiple of their net acceleration
constexpr float kDefaultRefineRatio = 1.0f;
// mixed path with jerk: evaluate in FP64 the pairs whose jerk scale
// m_j s_ij^-3/2 max_c |v_ij,c| exceeds this fraction of the i-particle's
// jerk (a few pairs per particle)
constexpr float kDefaultNearJerk = 0.0625f;
constexpr int kDefaultSmallLog2 = 27;    // 2^27 interactions: n_active x N_c
constexpr int64_t kMaxN = (int64_t)1 << 30;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Carve the workspace.  With base == nullptr only the size is computed.
// rows_per_j: partial rows per j-particle (a context's workspace holds
// kRowsPerJ + 1; the no-allocation evaluation's fixed buffer fewer).
size_t carve(int64_t n, int32_t C, char *base, Dev *d, int rows_per_j = nbk::kRowsPerJ + 1) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  Dev t{};
  t.n = n;
  t.C = C;
  t.nblk = (int32_t)((n + nbk::kScanBlock - 1) / nbk::kScanBlock);
  t.cap_active = n;
  t.rows_cap = (int64_t)rows_per_j * n + 4096;
  t.x = (double *)take(sizeof(double) * 3 * n);
  t.v = (double *)take(sizeof(double) * 3 * n);
  t.a = (double *)take(sizeof(double) * 3 * n);
  t.j = (double *)take(sizeof(double) * 3 * n);
  t.m = (double *)take(sizeof(double) * n);
  t.tick = (int64_t *)take(sizeof(int64_t) * n);
  t.level = (int32_t *)take(sizeof(int32_t) * n);
  t.cid = (int32_t *)take(sizeof(int32_t) * n);
  t.coff = (int64_t *)take(sizeof(int64_t) * (C + 1));
  t.eps2 = (double *)take(sizeof(double) * C);
  t.T = (int64_t *)take(sizeof(int64_t) * C);
  t.Tnext = (int64_t *)take(sizeof(int64_t) * C);
  t.Lthr = (int32_t *)take(sizeof(int32_t) * C);
  t.hist = (int32_t *)take(sizeof(int32_t) * C * nbk::kLevels);
  t.active = (int32_t *)take(sizeof(int32_t) * t.cap_active);
  t.act_off = (int32_t *)take(sizeof(int32_t) * (C + 1));
  t.blk_cnt = (int32_t *)take(sizeof(int32_t) * t.nblk);
  t.flag_cnt = (int32_t *)take(sizeof(int32_t) * t.nblk);
  t.blk_off = (int32_t *)take(sizeof(int32_t) * (t.nblk + 1));
  t.plan_c = (nbk::ClusterPlan *)take(sizeof(nbk::ClusterPlan) * C);
  t.plan_lpt = (nbk::ClusterPlan *)take(sizeof(nbk::ClusterPlan) * C);
  t.item_prefix = (int32_t *)take(sizeof(int32_t) * (C + 1));
  t.sum_prefix = (int32_t *)take(sizeof(int32_t) * (C + 1));
  t.partial = (double *)take(sizeof(double) * nbk::kRowStride * t.rows_cap);
  t.fsum = (double *)take(sizeof(double) * 6 * t.cap_active);
  t.rflag = (int32_t *)take(sizeof(int32_t) * t.cap_active);
  t.ref_i = (int32_t *)take(sizeof(int32_t) * t.cap_active);
  t.ref_k = (int32_t *)take(sizeof(int32_t) * t.cap_active);
  t.ref_off = (int32_t *)take(sizeof(int32_t) * (C + 1));
  t.theta = (float *)take(sizeof(float) * t.cap_active);
  t.pred = (void *)take((size_t)64 * n);
  t.pred_on = (int32_t *)take(sizeof(int32_t) * 4);
  t.work = (int32_t *)take(sizeof(int32_t) * 4);
  t.err = (int32_t *)take(sizeof(int32_t) * 4);
  t.sync = (int32_t *)take(sizeof(int32_t) * 4);
  t.vref = (double *)take(sizeof(double) * 3 * C);
  t.ctr = (int64_t *)take(sizeof(int64_t) * nbk::kCtrCount);
  t.eout = (double *)take(sizeof(double) * 9 * C);
  if (d) *d = t;
  return off;
}

bool is_pow2_step(double dt, int lmin, int lmax, int *level) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return false;
  int e;
  const double f = std::frexp(dt, &e);
  if (f != 0.5) return false;
  const int l = 1 - e;
  if (l < lmin || l > lmax) return false;
  if (level) *level = l;
  return true;
}

int validate_params(const nbody_params *p, int64_t n) {
  if (!p) return fail(NBODY_EINVAL, "params is NULL");
  if (n < 1 || n > kMaxN) return fail(NBODY_EINVAL, "n must be in [1, 2^30]");
  if (p->n_clusters < 1 || p->n_clusters > nbk::kMaxClusters)
    return fail(NBODY_EINVAL, "n_clusters must be in [1, 4096]");
  if (p->precision != NBODY_FP64 && p->precision != NBODY_MIXED &&
      p->precision != NBODY_MIXED_DS)
    return fail(NBODY_EINVAL, "unknown precision");
  const int C = p->n_clusters;
  if (p->cluster_offsets) {
    if (p->cluster_offsets[0] != 0 || p->cluster_offsets[C] != n)
      return fail(NBODY_EINVAL, "cluster_offsets must start at 0 and end at n");
    for (int c = 0; c < C; ++c)
      if (p->cluster_offsets[c + 1] <= p->cluster_offsets[c])
        return fail(NBODY_EINVAL, "cluster_offsets must be strictly increasing");
  } else if (C != 1) {
    return fail(NBODY_EINVAL, "cluster_offsets is NULL with n_clusters > 1");
  }
  if (!p->eps) return fail(NBODY_EINVAL, "eps is NULL");
  for (int c = 0; c < C; ++c)
    if (!(p->eps[c] >= 0.0) || !std::isfinite(p->eps[c]))
      return fail(NBODY_EINVAL, "eps must be finite and >= 0");
  if (!(p->eta > 0.0) || !std::isfinite(p->eta))
    return fail(NBODY_EINVAL, "eta must be > 0");
  if (!(p->eta_start > 0.0) || !std::isfinite(p->eta_start))
    return fail(NBODY_EINVAL, "eta_start must be > 0");
  if (p->level_min < 0 || p->level_max > nbk::kTickBits || p->level_min > p->level_max)
    return fail(NBODY_EINVAL, "need 0 <= level_min <= level_max <= 20");
  if (p->dt_shared != 0.0 && !is_pow2_step(p->dt_shared, p->level_min, p->level_max, nullptr))
    return fail(NBODY_EINVAL, "dt_shared must be 0 or a power of two within the level range");
  if (p->field) {
    const nbody_field &f = *p->field;
    const double all[] = {f.bulge_m, f.bulge_b, f.disk_m, f.disk_a, f.disk_b,
                          f.halo_m, f.halo_a, f.halo_gamma, f.halo_rc};
    for (double q : all)
      if (!std::isfinite(q)) return fail(NBODY_EINVAL, "field parameters must be finite");
    if (f.bulge_m < 0.0 || f.disk_m < 0.0 || f.halo_m < 0.0)
      return fail(NBODY_EINVAL, "field masses must be >= 0");
    if (f.bulge_m > 0.0 && !(f.bulge_b > 0.0))
      return fail(NBODY_EINVAL, "field bulge_b must be > 0");
    if (f.disk_m > 0.0 && (!(f.disk_a >= 0.0) || !(f.disk_b > 0.0)))
      return fail(NBODY_EINVAL, "field disk needs disk_a >= 0 and disk_b > 0");
    if (f.halo_m > 0.0 && (!(f.halo_a > 0.0) || !(f.halo_gamma > 0.0) || !(f.halo_rc > 0.0)))
      return fail(NBODY_EINVAL, "field halo needs halo_a, halo_gamma, halo_rc > 0");
  }
  return NBODY_OK;
}

// Device copy of the external field, with the halo's mass inside the
// cut-off and the constant of its inner potential.
nbk::Field make_field(const nbody_field *f) {
  nbk::Field d{};
  if (!f || (f->bulge_m == 0.0 && f->disk_m == 0.0 && f->halo_m == 0.0)) return d;
  d.on = 1;
  d.bm = f->bulge_m;
  d.bb = f->bulge_b;
  d.dm = f->disk_m;
  d.da = f->disk_a;
  d.db = f->disk_b;
  d.hm = f->halo_m;
  d.ha = f->halo_a;
  d.hg = f->halo_gamma;
  d.hrc = f->halo_rc;
  if (d.hm != 0.0) {
    const double sc = d.hrc / d.ha, scg = std::pow(sc, d.hg);
    d.hmc = d.hm * sc * scg / (1.0 + scg);
    d.hpc = -d.hmc / d.hrc - d.hm / (d.hg * d.ha) * std::log1p(scg);
  }
  return d;
}

int device_present(int *dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return fail(NBODY_ENODEV, "no HIP device");
  if (hipGetDevice(dev) != hipSuccess) return fail(NBODY_ENODEV, "hipGetDevice failed");
  return NBODY_OK;
}

// FP32 pair arithmetic (either mixed form)
bool is_mixed(int precision) {
  return precision == NBODY_MIXED || precision == NBODY_MIXED_DS;
}

nbody_tuning default_tuning(int precision) {
  nbody_tuning t;
  std::memset(&t, 0, sizeof t);
  // measured on MI355X at N = 2^18 and 2^20: the mixed loop with FP64
  // differences runs fastest with one i per lane fed from scalar registers
  // (its FP64 records as SGPR operands), the double-single one with one i
  // per lane from LDS (more waves in flight), the FP64 loop with two i per
  // lane from scalar registers
  t.variant = precision == NBODY_MIXED      ? NBODY_VARIANT_S1
              : precision == NBODY_MIXED_DS ? NBODY_VARIANT_K1
                                            : NBODY_VARIANT_S2;
  t.use_graph = NBODY_GRAPH_ON;
  t.steps_per_launch = 16;
  t.min_split_j = 256;
  t.refine_ratio = is_mixed(precision) ? kDefaultRefineRatio : -1.0f;
  t.near_jerk = is_mixed(precision) ? kDefaultNearJerk : -1.0f;
  t.small_log2 = kDefaultSmallLog2;
  const int K = (t.variant == NBODY_VARIANT_K2) ? 2 : 1;
  for (int b = 0; b < NBODY_TUNE_BUCKETS; ++b) {
    // one i-tile covers the bucket [2^b, 2^(b+1)) when possible
    int64_t cover = ((int64_t)2 << b) / K;
    if (b == 0) cover = 1;
    if (cover < 1) cover = 1;
    int P = 1;
    while (P < cover && P < 256) P <<= 1;
    t.i_slots[b] = P;
    // from 2^16 active particles on, split j as finely as the partial rows
    // allow: 2 MB chunks at N = 2^20, which each XCD's L2 holds while all
    // resident workgroups stream them
    t.target_items[b] = b >= 16 ? 131072 : 2048;
  }
  return t;
}

int map_err_bits(int bits) {
  if (bits & nbk::kErrDomain)
    return fail(NBODY_EDOMAIN, "eps == 0 and two distinct particles coincide");
  if (bits & nbk::kErrNonFinite)
    return fail(NBODY_ENONFINITE, "non-finite acceleration, jerk or state");
  if (bits & nbk::kErrIndex)
    return fail(NBODY_EINDEX, "i index out of range or i_active not grouped by cluster");
  if (bits) return fail(NBODY_EINVAL, "invalid state");
  return NBODY_OK;
}

}  // namespace

struct nbody_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t cap = nullptr;      // private stream used only for capture
  int64_t n = 0;
  int32_t C = 1;
  int prec = NBODY_FP64;
  double eta = 0, eta_start = 0, dt_shared = 0;
  int lmin = 0, lmax = 0;
  std::vector<int64_t> coff;
  std::vector<int64_t> T_host;    // cluster times known to the host
  Dev d{};
  nbody_tuning tune{};
  int K = 1;
  bool sb = false;                // broadcast kernel for large evaluations
  int Ka = 1;                     // the same two for the acceleration-only
  bool sba = false;               // evaluations (tuning acc_variant)
  bool step_sb_only = false;      // mixed block steps: the broadcast kernel
                                  // provably takes every main item
  int grid_state = 0, grid_raw = 0, grid_pot = 0, grid_sb = 0;
  int grid_ref_state = 0, grid_ref_raw = 0;   // FP64 K = 1 re-evaluation
  int grid_small = 0;             // FP64, the context's K: small mixed block steps
  int grid_rec = 0, grid_acc_rec = 0;   // record-only kernels
  // acceleration-only kernels (symplectic drivers, nbody_accel)
  int grid_acc_state = 0, grid_acc_raw = 0, grid_acc_sb = 0;
  int grid_ref_acc_state = 0, grid_ref_acc_raw = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_steps = 0;
  int64_t *pinned = nullptr;      // host pinned readback words (32 x int64)
  // profiling: event pairs around force-kernel launches
  bool profiling = false;
  std::vector<hipEvent_t> ev;     // 2 * kEvPairs events
  std::vector<int> ev_tag;        // kind of launch each recorded pair brackets
  int ev_used = 0;                // pairs recorded since the last harvest
  double prof_ms[2] = {0.0, 0.0};         // [0] precision's own kernel, [1] FP64 re-evaluation
  int64_t prof_launches[2] = {0, 0};
};

namespace {

nbk::Tuning device_tuning(const nbody_ctx *c, int K) {
  nbk::Tuning t{};
  for (int b = 0; b < nbk::kBuckets; ++b) {
    t.i_slots[b] = c->tune.i_slots[b];
    t.target_items[b] = c->tune.target_items[b];
  }
  t.min_split_j = c->tune.min_split_j;
  t.K = K;
  t.small_work = c->tune.small_log2 < 0 ? -1 : (int64_t)1 << c->tune.small_log2;
  return t;
}

int mode_of(const nbody_ctx *c) {
  return c->prec == NBODY_MIXED ? nbk::kModeMixed64
         : c->prec == NBODY_MIXED_DS ? nbk::kModeMixed : nbk::kModeFP64;
}

int acc_mode_of(const nbody_ctx *c) {
  return c->prec == NBODY_MIXED ? nbk::kModeMixed64Acc
         : c->prec == NBODY_MIXED_DS ? nbk::kModeMixedAcc : nbk::kModeFP64Acc;
}

void drop_graph(nbody_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->graph_steps = 0;
}

int refresh_grids(nbody_ctx *c) {
  const int v = c->tune.variant;
  c->K = (v == NBODY_VARIANT_K2 || v == NBODY_VARIANT_S2) ? 2 : 1;
  c->sb = (v == NBODY_VARIANT_S1 || v == NBODY_VARIANT_S2);
  const int va = c->tune.acc_variant ? c->tune.acc_variant : v;
  c->Ka = (va == NBODY_VARIANT_K2 || va == NBODY_VARIANT_S2) ? 2 : 1;
  c->sba = (va == NBODY_VARIANT_S1 || va == NBODY_VARIANT_S2);
  // A mixed block step's records are always built, and the record kernel
  // hands the main items to the broadcast kernel when every cluster with
  // main work has kWG i-slots.  With small steps routed to FP64, only the
  // buckets of active counts that some cluster does not route there can
  // hold main work (more than kSmallStep active particles, and more than
  // small_work interactions in the largest cluster); when the i-slots of
  // those buckets are all kWG the workgroup kernel's launch would only
  // return: it is not enqueued.
  c->step_sb_only = c->sb && is_mixed(c->prec) && c->tune.small_log2 >= 0;
  if (c->step_sb_only) {
    int64_t nmax = c->n;
    if ((int64_t)c->coff.size() == (int64_t)c->C + 1) {
      nmax = 0;
      for (int k = 0; k < c->C; ++k) nmax = std::max(nmax, c->coff[k + 1] - c->coff[k]);
    }
    const int64_t sw = (int64_t)1 << c->tune.small_log2;
    for (int b = 0; b < nbk::kBuckets; ++b) {
      const int64_t lo = (int64_t)1 << b;
      const int64_t hi = b + 1 < nbk::kBuckets ? 2 * lo - 1 : nmax;   // last bucket: the rest
      if (lo > nmax) break;                          // no cluster that large
      const bool all_small = hi <= nbk::kSmallStep || hi * nmax <= sw;
      if (!all_small && c->tune.i_slots[b] != nbk::kWG) c->step_sb_only = false;
    }
  }
  c->grid_sb = c->sb ? nbk::force_sb_grid_size(mode_of(c), c->K, c->device) : 1;
  c->grid_acc_sb = c->sba ? nbk::force_sb_grid_size(acc_mode_of(c), c->Ka, c->device) : 1;
  c->grid_acc_state = nbk::force_grid_size(acc_mode_of(c), nbk::kSrcState, c->Ka, c->device);
  c->grid_acc_raw = nbk::force_grid_size(acc_mode_of(c), nbk::kSrcRaw, c->Ka, c->device);
  c->grid_ref_acc_state = nbk::force_grid_size(nbk::kModeFP64Acc, nbk::kSrcState, 1, c->device);
  c->grid_ref_acc_raw = nbk::force_grid_size(nbk::kModeFP64Acc, nbk::kSrcRaw, 1, c->device);
  c->grid_state = nbk::force_grid_size(mode_of(c), nbk::kSrcState, c->K, c->device);
  c->grid_raw = nbk::force_grid_size(mode_of(c), nbk::kSrcRaw, c->K, c->device);
  c->grid_pot = nbk::force_grid_size(nbk::kModePot, nbk::kSrcState, 1, c->device);
  c->grid_ref_state = nbk::force_grid_size(nbk::kModeFP64, nbk::kSrcState, 1, c->device);
  c->grid_ref_raw = nbk::force_grid_size(nbk::kModeFP64, nbk::kSrcRaw, 1, c->device);
  c->grid_small = nbk::force_grid_size(nbk::kModeFP64, nbk::kSrcState, c->K, c->device);
  c->grid_rec = nbk::force_grid_size(mode_of(c), nbk::kSrcRec, c->K, c->device);
  c->grid_acc_rec = nbk::force_grid_size(acc_mode_of(c), nbk::kSrcRec, c->Ka, c->device);
  if (c->grid_state < 1 || c->grid_raw < 1 || c->grid_pot < 1 || c->grid_ref_state < 1 ||
      c->grid_ref_raw < 1 || c->grid_small < 1 || c->grid_rec < 1 || c->grid_acc_rec < 1 ||
      c->grid_sb < 1 || c->grid_acc_sb < 1 || c->grid_acc_state < 1 ||
      c->grid_acc_raw < 1 || c->grid_ref_acc_state < 1 || c->grid_ref_acc_raw < 1)
    return fail(NBODY_EHIP, "could not size the force kernel grid");
  return NBODY_OK;
}

int harvest_events(nbody_ctx *c);

// Block steps of one cluster whose compaction also plans build their j
// records in the compaction too (one launch fewer per step).
bool rec_in_compact(const nbody_ctx *c) { return nbk::plan_fused(c->d); }

// Launch the force kernel, bracketed by timing events when profiling.
// rec_kind >= 0 (a PlanKind): build the evaluation's j records first when its
// active set is large, and let the broadcast kernel take it when enabled.
int force_launch(nbody_ctx *c, int mode, int src, int K, const nbk::RawSrc *raw,
                 const int32_t *list, int grid, hipStream_t s, int rec_kind = -1,
                 nbk::NearSpec nr = nbk::NearSpec{nbk::kNearNone, 0.0f}) {
  const bool prof = c->profiling && s == c->stream;
  const bool use_pred = rec_kind >= 0;
  const bool mixed_step = rec_kind == nbk::kPlanStep && nbk::mode_mixed(mode) &&
                          !nbk::mode_acc_only(mode);
  // clusters of a mixed block step with few active particles run in FP64
  // (unless that routing is off)
  const bool small = mixed_step && c->tune.small_log2 >= 0;
  // evaluations whose records are always built (mixed block steps beyond
  // the small ones, whole-state evaluations) use the record-only kernel
  const bool rec_only = mixed_step || rec_kind == nbk::kPlanState;
  const bool sb = nbk::mode_acc_only(mode) ? c->sba : c->sb;
  const bool sb_only = mixed_step && c->step_sb_only;
  if (use_pred && !(rec_kind == nbk::kPlanStep && rec_in_compact(c)))
    NB_HIP(nbk::launch_records(c->d, mode, rec_kind, raw, sb, rec_only, sb_only, s));
  if (prof && c->ev_used == kEvPairs) {
    int rc = harvest_events(c);
    if (rc) return rc;
  }
  if (prof) NB_HIP(hipEventRecord(c->ev[2 * c->ev_used], s));
  if (!sb_only)
    NB_HIP(nbk::launch_force(c->d, mode, rec_only ? nbk::kSrcRec : src, K, raw, list,
                              use_pred ? nbk::kRoleMain : nbk::kRoleAlways, nr,
                              rec_only ? (nbk::mode_acc_only(mode) ? c->grid_acc_rec
                                                                   : c->grid_rec)
                                       : grid,
                              s));
  if (use_pred && sb)
    NB_HIP(nbk::launch_force_sb(c->d, mode, K, raw, list, nr,
                                nbk::mode_acc_only(mode) ? c->grid_acc_sb : c->grid_sb, s));
  if (small)
    NB_HIP(nbk::launch_force(c->d, nbk::kModeFP64, src, K, raw, list, nbk::kRoleSmall,
                             nbk::NearSpec{nbk::kNearNone, 0.0f}, c->grid_small, s));
  if (prof) {
    NB_HIP(hipEventRecord(c->ev[2 * c->ev_used + 1], s));
    // the potential kernel (energy diagnostics) is not counted; FP64 launches
    // of a mixed context are its re-evaluations
    const bool fp64 = mode == nbk::kModeFP64 || mode == nbk::kModeFP64Acc;
    c->ev_tag[c->ev_used] =
        (mode == nbk::kModePot) ? -1 : ((fp64 && is_mixed(c->prec)) ? 1 : 0);
    ++c->ev_used;
  }
  return NBODY_OK;
}

// Wait for the recorded pairs and add their durations.
int harvest_events(nbody_ctx *c) {
  if (!c->ev_used) return NBODY_OK;
  NB_HIP(hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->ev_used; ++k) {
    const int tag = c->ev_tag[k];
    if (tag < 0) continue;
    float ms = 0.0f;
    NB_HIP(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    c->prof_ms[tag] += ms;
    c->prof_launches[tag] += 1;
  }
  c->ev_used = 0;
  return NBODY_OK;
}

float refine_ratio(const nbody_ctx *c) {
  return (is_mixed(c->prec) && c->tune.refine_ratio > 0.0f) ? c->tune.refine_ratio : 0.0f;
}

// Near pairs of a mixed evaluation with jerk, from the given threshold
// source, when the context's precision and tuning use them.
nbk::NearSpec near_spec(const nbody_ctx *c, int mode, int src) {
  nbk::NearSpec nr;
  nr.c = c->tune.near_jerk;
  const bool on = is_mixed(c->prec) && nr.c > 0.0f && !nbk::mode_acc_only(mode) &&
                  mode != nbk::kModePot && mode != nbk::kModeFP64;
  nr.src = on ? src : nbk::kNearNone;
  if (!on) nr.c = 0.0f;
  // block steps take the estimate from the stored jerk of the particle's
  // previous step: half the threshold, and a stale bound of kNearStaleState
  // instead of kNearStale, give the same effective threshold (at most
  // 2 near_jerk times the jerk found) while tolerating a jerk that fell
  // by up to 4x over the step
  if (nr.src == nbk::kNearState) nr.c *= 0.5f;
  return nr;
}

// Sum the partial rows into fsum and, on the mixed path, re-evaluate the
// flagged entries with the FP64 kernel (a second plan over the flagged list).
// nr: where the evaluation's near-pair thresholds came from (the flags test
// them against the jerk found).  corr (block steps): the flagged entries are
// appended (one cluster), and the re-evaluation's final launch applies the
// corrector to every active particle.
int sum_and_refine(nbody_ctx *c, const int32_t *list, int64_t na_host, const nbk::RawSrc *raw,
                   hipStream_t s, bool acc_only, nbk::NearSpec nr,
                   const nbk::CorrectSpec *corr = nullptr) {
  const float ratio = refine_ratio(c);
  const nbk::Tuning t1 = device_tuning(c, 1);
  const bool api = raw != nullptr;
  const int ref_kind = api ? nbk::kPlanApiRefine : nbk::kPlanRefine;
  const int64_t api_nj = api ? raw->n_j : 0;
  NB_HIP(nbk::launch_sum_and_flag(c->d, list, na_host, ratio, nr, false, t1, ref_kind, api_nj,
                                  corr != nullptr, s));
  if (ratio <= 0.0f) return NBODY_OK;
  if (!nbk::plan_fused(c->d))
    NB_HIP(nbk::launch_plan(c->d, t1, ref_kind, api_nj, false, s));
  const int grid = acc_only ? (api ? c->grid_ref_acc_raw : c->grid_ref_acc_state)
                            : (api ? c->grid_ref_raw : c->grid_ref_state);
  int rc = force_launch(c, acc_only ? nbk::kModeFP64Acc : nbk::kModeFP64,
                        api ? nbk::kSrcRaw : nbk::kSrcState, 1, raw, c->d.ref_i, grid, s);
  if (rc) return rc;
  NB_HIP(nbk::launch_refine_finalize(c->d, corr, s));
  return NBODY_OK;
}

// One mixed evaluation with jerk when no jerk estimate is at hand (initial
// state, full re-evaluations, nbody_forces): a first pass without near pairs
// gives each entry's jerk, from which the second pass takes its near-pair
// thresholds.  `launch` enqueues the force launch(es) of one pass (the plan
// and the records stay valid; the item counters are reset in between).
template <class F>
int two_pass(nbody_ctx *c, const int32_t *list, int64_t na_host, const nbk::RawSrc *raw,
             hipStream_t s, int mode, F launch) {
  const nbk::NearSpec first = near_spec(c, mode, nbk::kNearNone);
  const nbk::NearSpec second = near_spec(c, mode, nbk::kNearList);
  int rc = launch(first);
  if (rc) return rc;
  if (second.src == nbk::kNearList) {
    const nbk::Tuning t1 = device_tuning(c, 1);
    NB_HIP(nbk::launch_sum_and_flag(c->d, list, na_host, 0.0f, second, true, t1, 0, 0, false,
                                    s));
    NB_HIP(nbk::launch_fill32(c->d.work, 0, 2, s));
    if ((rc = launch(second))) return rc;
  }
  return sum_and_refine(c, list, na_host, raw, s, nbk::mode_acc_only(mode), second);
}

// One Hermite block step for every cluster, enqueued on s.  The near-pair
// thresholds come from each active particle's stored jerk.
int enqueue_block_step(nbody_ctx *c, hipStream_t s) {
  const nbk::Tuning t = device_tuning(c, c->K);
  const bool allow_small = is_mixed(c->prec);
  const bool rc_records = rec_in_compact(c);
  NB_HIP(nbk::launch_compact(c->d, t, allow_small, rc_records ? mode_of(c) : -1, c->sb,
                             rc_records && is_mixed(c->prec) && c->step_sb_only, s));
  if (!nbk::plan_fused(c->d))
    NB_HIP(nbk::launch_plan(c->d, t, nbk::kPlanStep, 0, allow_small, s));
  const nbk::NearSpec nr = near_spec(c, mode_of(c), nbk::kNearState);
  int rc = force_launch(c, mode_of(c), nbk::kSrcState, c->K, nullptr, c->d.active,
                        c->grid_state, s, nbk::kPlanStep, nr);
  if (rc) return rc;
  // with re-evaluation: sums and flags, the FP64 pass, then its final
  // launch corrects every active particle; without: the corrector sums the
  // rows itself
  if (refine_ratio(c) > 0.0f) {
    const nbk::CorrectSpec cs{c->eta, c->dt_shared, c->lmin, c->lmax};
    return sum_and_refine(c, c->d.active, -1, nullptr, s, false, nr, &cs);
  }
  NB_HIP(nbk::launch_correct(c->d, c->eta, c->dt_shared, c->lmin, c->lmax, s));
  return NBODY_OK;
}

int ensure_graph(nbody_ctx *c) {
  const int steps = c->tune.steps_per_launch;
  if (c->gexec && c->graph_steps == steps) return NBODY_OK;
  drop_graph(c);
  NB_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
  int rc = NBODY_OK;
  for (int k = 0; k < steps && rc == NBODY_OK; ++k) rc = enqueue_block_step(c, c->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (rc != NBODY_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(NBODY_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  c->graph = g;
  NB_HIP(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  c->graph_steps = steps;
  return NBODY_OK;
}

// Wait for the stream, then fetch counters and error bits into pinned.
int readback(nbody_ctx *c) {
  NB_HIP(hipMemcpyAsync(c->pinned, c->d.ctr, sizeof(int64_t) * nbk::kCtrCount,
                        hipMemcpyDeviceToHost, c->stream));
  NB_HIP(hipMemcpyAsync(c->pinned + 16, c->d.err, sizeof(int32_t), hipMemcpyDeviceToHost,
                        c->stream));
  NB_HIP(hipStreamSynchronize(c->stream));
  return NBODY_OK;
}

int take_error(nbody_ctx *c) {
  const int bits = *(const int32_t *)(c->pinned + 16);
  if (!bits) return NBODY_OK;
  NB_HIP(nbk::launch_fill32(c->d.err, 0, 1, c->stream));
  NB_HIP(hipStreamSynchronize(c->stream));
  *(int32_t *)(c->pinned + 16) = 0;
  return map_err_bits(bits);
}

int full_evaluation_into_state(nbody_ctx *c) {
  // initial forces: every particle active, predicted to its own time
  const nbk::Tuning t = device_tuning(c, c->K);
  if (c->prec == NBODY_MIXED) NB_HIP(nbk::launch_vref(c->d, nullptr, c->stream));
  NB_HIP(nbk::launch_all_active(c->d, t, c->stream));
  if (c->C > 1) NB_HIP(nbk::launch_plan(c->d, t, nbk::kPlanState, 0, false, c->stream));
  // all particles start at T = T_next = 0, so the re-evaluation plan
  // (predicting to T_next) sees the same positions
  int rc = two_pass(c, c->d.active, -1, nullptr, c->stream, mode_of(c),
                    [&](nbk::NearSpec nr) {
                      return force_launch(c, mode_of(c), nbk::kSrcState, c->K, nullptr,
                                          c->d.active, c->grid_state, c->stream,
                                          nbk::kPlanState, nr);
                    });
  if (rc) return rc;
  NB_HIP(nbk::launch_init_levels(c->d, c->eta_start, c->dt_shared, c->lmin, c->lmax,
                                 c->stream));
  return NBODY_OK;
}

// t_end of nbody_step / nbody_step_blocks in ticks, validated.
int check_t_end(const nbody_ctx *c, double t_end, int64_t *tend_out) {
  if (!std::isfinite(t_end) || t_end < 0.0) return fail(NBODY_EINVAL, "t_end must be finite and >= 0");
  const double tt = t_end * (double)(1 << nbk::kTickBits);
  if (tt > 9.0e15 || tt != std::floor(tt))
    return fail(NBODY_EINVAL, "t_end must be a multiple of 2^-20");
  const int64_t tend = (int64_t)tt;
  const int64_t dtmax = (int64_t)1 << (nbk::kTickBits - c->lmin);
  if (tend % dtmax) return fail(NBODY_EINVAL, "t_end must be a multiple of 2^-level_min");
  for (int k = 0; k < c->C; ++k)
    if (tend < c->T_host[k]) return fail(NBODY_EINVAL, "t_end is earlier than the current time");
  *tend_out = tend;
  return NBODY_OK;
}

// nbody_forces / nbody_accel: the caller's j arrays, chunks of at most
// cap_active i entries.
int api_forces(nbody_ctx *c, bool acc_only, const int32_t *i_active, int64_t n_active,
               const double *xj, const double *vj, const double *mj, int64_t n_j, double *acc,
               double *jerk) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  if (n_active < 0) return fail(NBODY_EINVAL, "n_active < 0");
  if (n_active == 0) return NBODY_OK;
  if (!i_active || !xj || !mj || !acc) return fail(NBODY_EINVAL, "NULL array argument");
  if (n_j < 1 || n_j > kMaxN) return fail(NBODY_EINVAL, "n_j must be in [1, 2^30]");
  if (c->C > 1 && n_j != c->n)
    return fail(NBODY_EINVAL, "with several clusters n_j must equal the context's n");
  const int mode = acc_only ? acc_mode_of(c) : mode_of(c);
  const int grid = acc_only ? c->grid_acc_raw : c->grid_raw;
  const int K = acc_only ? c->Ka : c->K;
  const nbk::Tuning t = device_tuning(c, K);
  const int64_t cap = c->d.cap_active;
  for (int64_t k0 = 0; k0 < n_active; k0 += cap) {
    nbk::RawSrc r;
    r.x = xj;
    r.v = vj;
    r.m = mj;
    r.n_j = (c->C == 1) ? n_j : 0;
    r.i_active = i_active + k0;
    r.n_active = (n_active - k0 < cap) ? n_active - k0 : cap;
    r.acc = acc + 3 * k0;
    r.jerk = jerk ? jerk + 3 * k0 : nullptr;
    NB_HIP(nbk::launch_api_group(c->d, r, t, c->stream));
    if (c->prec == NBODY_MIXED && !acc_only) NB_HIP(nbk::launch_vref(c->d, &r, c->stream));
    if (c->C > 1) NB_HIP(nbk::launch_plan(c->d, t, nbk::kPlanApi, r.n_j, false, c->stream));
    int rc = two_pass(c, r.i_active, r.n_active, &r, c->stream, mode, [&](nbk::NearSpec nr) {
      return force_launch(c, mode, nbk::kSrcRaw, K, &r, r.i_active, grid, c->stream,
                          nbk::kPlanApi, nr);
    });
    if (rc) return rc;
    NB_HIP(nbk::launch_api_finalize(c->d, r, c->stream));
  }
  return NBODY_OK;
}

}  // namespace

extern "C" {

size_t nbody_workspace_bytes(const nbody_params *p, int64_t n) {
  if (validate_params(p, n) != NBODY_OK) return 0;
  return carve(n, p->n_clusters, nullptr, nullptr);
}

int nbody_init(nbody_ctx **out, const nbody_params *p, int64_t n, const double *m,
               const double *x, const double *v) {
  if (!out) return fail(NBODY_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_params(p, n);
  if (rc) return rc;
  if (!m || !x || !v) return fail(NBODY_EINVAL, "m, x or v is NULL");
  if (!p->workspace) return fail(NBODY_EINVAL, "workspace is NULL");
  if ((uintptr_t)p->workspace % kAlign)
    return fail(NBODY_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = carve(n, p->n_clusters, nullptr, nullptr);
  if (p->workspace_bytes < need)
    return fail(NBODY_ENOMEM, "workspace smaller than nbody_workspace_bytes()");
  int dev = 0;
  rc = device_present(&dev);
  if (rc) return rc;

  nbody_ctx *c = new (std::nothrow) nbody_ctx();
  if (!c) return fail(NBODY_EINVAL, "out of host memory");
  c->device = dev;
  c->stream = (hipStream_t)p->stream;
  c->n = n;
  c->C = p->n_clusters;
  c->prec = p->precision;
  c->eta = p->eta;
  c->eta_start = p->eta_start;
  c->dt_shared = p->dt_shared;
  c->lmin = p->level_min;
  c->lmax = p->level_max;
  c->coff.resize(c->C + 1);
  if (p->cluster_offsets)
    std::memcpy(c->coff.data(), p->cluster_offsets, sizeof(int64_t) * (c->C + 1));
  else {
    c->coff[0] = 0;
    c->coff[1] = n;
  }
  c->T_host.assign(c->C, 0);
  carve(n, c->C, (char *)p->workspace, &c->d);
  c->d.fld = make_field(p->field);
  c->tune = default_tuning(c->prec);
  auto bail = [&](int code) {
    nbody_destroy(c);
    return code;
  };
  if ((rc = refresh_grids(c))) return bail(rc);
  if (hipHostMalloc((void **)&c->pinned, 32 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
    return bail(fail(NBODY_EHIP, "hipHostMalloc failed"));
  std::memset(c->pinned, 0, 32 * sizeof(int64_t));
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(NBODY_EHIP, "hipStreamCreate failed"));
  std::vector<double> eps2(c->C);
  for (int k = 0; k < c->C; ++k) eps2[k] = p->eps[k] * p->eps[k];
  if (hipMemcpyAsync(c->d.coff, c->coff.data(), sizeof(int64_t) * (c->C + 1),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d.eps2, eps2.data(), sizeof(double) * c->C,
                     hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return bail(fail(NBODY_EHIP, "upload of cluster tables failed"));
  if (nbk::launch_init_state(c->d, m, x, v, c->stream) != hipSuccess)
    return bail(fail(NBODY_EHIP, "init kernel launch failed"));
  if ((rc = full_evaluation_into_state(c))) return bail(rc);
  if ((rc = readback(c))) return bail(rc);
  if ((rc = take_error(c))) return bail(rc);
  *out = c;
  return NBODY_OK;
}

int nbody_forces(nbody_ctx *c, const int32_t *i_active, int64_t n_active, const double *xj,
                 const double *vj, const double *mj, int64_t n_j, double *acc, double *jerk) {
  if (c && n_active > 0 && (!vj || !jerk)) return fail(NBODY_EINVAL, "NULL array argument");
  return api_forces(c, false, i_active, n_active, xj, vj, mj, n_j, acc, jerk);
}

int nbody_accel(nbody_ctx *c, const int32_t *i_active, int64_t n_active, const double *xj,
                const double *mj, int64_t n_j, double *acc) {
  return api_forces(c, true, i_active, n_active, xj, nullptr, mj, n_j, acc, nullptr);
}

int nbody_step_symplectic(nbody_ctx *c, int scheme, double h, int64_t n_steps,
                          int64_t *n_interactions) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  if (scheme != NBODY_LEAPFROG && scheme != NBODY_SYMPLECTIC6)
    return fail(NBODY_EINVAL, "unknown symplectic scheme");
  if (n_steps < 0) return fail(NBODY_EINVAL, "n_steps < 0");
  const double ht = h * (double)(1 << nbk::kTickBits);
  if (!(h > 0.0) || !std::isfinite(h) || ht != std::floor(ht) || ht > 9.0e15)
    return fail(NBODY_EINVAL, "h must be a positive multiple of 2^-20");
  const int64_t hticks = (int64_t)ht;
  const int64_t dtmax = (int64_t)1 << (nbk::kTickBits - c->lmin);
  if (n_steps > (int64_t)9.0e15 / hticks) return fail(NBODY_EINVAL, "n_steps * h too large");
  const int64_t span = n_steps * hticks;
  if (span % dtmax)
    return fail(NBODY_EINVAL, "n_steps * h must be a multiple of 2^-level_min");
  int rc = readback(c);
  if (rc) return rc;
  if ((rc = take_error(c))) return rc;
  if (n_interactions) *n_interactions = 0;
  if (n_steps == 0) return NBODY_OK;
  // stage weights: one leapfrog stage, or the symmetric seven-stage
  // composition of sixth order (w3 w2 w1 w0 w1 w2 w3, w0 = 1 - 2 (w1 + w2 + w3))
  std::vector<double> w;
  if (scheme == NBODY_LEAPFROG) {
    w = {1.0};
  } else {
    const double w1 = -1.17767998417887, w2 = 0.235573213359357, w3 = 0.784513610477560;
    const double w0 = 1.0 - 2.0 * (w1 + w2 + w3);
    w = {w3, w2, w1, w0, w1, w2, w3};
  }
  const int mode = acc_mode_of(c);
  const nbk::Tuning t = device_tuning(c, c->Ka);
  // with one cluster the kernel before each evaluation (the all-active
  // setup, then every kick-drift) writes its plan
  NB_HIP(nbk::launch_all_active(c->d, t, c->stream));
  auto evaluate = [&](hipStream_t s) -> int {
    if (c->C > 1) NB_HIP(nbk::launch_plan(c->d, t, nbk::kPlanState, 0, false, s));
    int r = force_launch(c, mode, nbk::kSrcState, c->Ka, nullptr, c->d.active, c->grid_acc_state,
                         s, nbk::kPlanState);
    if (r) return r;
    return sum_and_refine(c, c->d.active, -1, nullptr, s, /*acc_only=*/true,
                          nbk::NearSpec{nbk::kNearNone, 0.0f});
  };
  // one step: every stage kicks (merging the previous stage's half kick),
  // drifts and evaluates; returns the half kick still owed
  auto enqueue_step = [&](hipStream_t s, double pending, bool check, double *owed) -> int {
    for (double wk : w) {
      const double cw = wk * h;
      NB_HIP(nbk::launch_sym_kick_drift(c->d, pending + 0.5 * cw, cw, check, t, s));
      check = false;
      int r = evaluate(s);
      if (r) return r;
      pending = 0.5 * cw;
    }
    *owed = pending;
    return NBODY_OK;
  };
  // the state's acceleration was taken at predicted positions: evaluate
  // at the current ones first
  if ((rc = evaluate(c->stream))) return rc;
  double pending = 0.0;
  if ((rc = enqueue_step(c->stream, 0.0, true, &pending))) return rc;
  const int64_t evals = 1 + n_steps * (int64_t)w.size();
  // the remaining steps are identical: capture one as a HIP graph and
  // replay it (eager launches when profiling, or for a few steps)
  const int64_t rest = n_steps - 1;
  if (rest >= 4 && !c->profiling) {
    NB_HIP(hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    double owed = 0.0;
    rc = enqueue_step(c->cap, pending, false, &owed);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (rc != NBODY_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : fail(NBODY_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess)
      return fail(NBODY_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    for (int64_t st = 0; st < rest && rc == NBODY_OK; ++st) {
      const hipError_t el = hipGraphLaunch(ge, c->stream);
      if (el != hipSuccess) rc = fail(NBODY_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(el));
      // bound the host's lead over the device on long runs
      if (rc == NBODY_OK && (st & 63) == 63) rc = readback(c);
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipGraphExecDestroy(ge);
    if (rc) return rc;
    pending = owed;
  } else {
    for (int64_t st = 0; st < rest; ++st) {
      if ((rc = enqueue_step(c->stream, pending, false, &pending))) return rc;
      if ((st & 63) == 63 && (rc = readback(c))) return rc;
    }
  }
  NB_HIP(nbk::launch_sym_kick(c->d, pending, c->stream));
  NB_HIP(nbk::launch_sym_advance(c->d, span, c->stream));
  for (int k = 0; k < c->C; ++k) c->T_host[k] += span;
  // leave a consistent Hermite state: a, jerk and levels at the new positions
  if ((rc = full_evaluation_into_state(c))) return rc;
  if ((rc = readback(c))) return rc;
  if ((rc = take_error(c))) return rc;
  if (n_interactions) {
    int64_t pairs = 0;
    for (int k = 0; k < c->C; ++k) {
      const int64_t nc = c->coff[k + 1] - c->coff[k];
      pairs += nc * nc;
    }
    *n_interactions = evals * pairs;
  }
  return NBODY_OK;
}

int nbody_step(nbody_ctx *c, double t_end, int64_t *n_block_steps, int64_t *n_interactions) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  int64_t tend = 0;
  int rc = check_t_end(c, t_end, &tend);
  if (rc) return rc;
  rc = readback(c);
  if (rc) return rc;
  if ((rc = take_error(c))) return rc;
  const int64_t steps0 = c->pinned[nbk::kCtrSteps], inter0 = c->pinned[nbk::kCtrInter];
  NB_HIP(nbk::launch_set_word64(c->d.ctr + nbk::kCtrTend, tend, c->stream));
  // an upper bound on block steps: every step moves some cluster by >= 1 tick
  int64_t remaining = 0;
  for (int k = 0; k < c->C; ++k) remaining += tend - c->T_host[k];
  int64_t launches = 0;
  const int64_t max_launches = remaining / (c->tune.steps_per_launch > 0 ? c->tune.steps_per_launch : 1) + 2;
  while (remaining > 0) {
    // the records' reference velocities follow the clusters' bulk motion
    if (c->prec == NBODY_MIXED) NB_HIP(nbk::launch_vref(c->d, nullptr, c->stream));
    if (c->tune.use_graph == NBODY_GRAPH_ON && !c->profiling) {
      if ((rc = ensure_graph(c))) return rc;
      NB_HIP(hipGraphLaunch(c->gexec, c->stream));
    } else {
      for (int k = 0; k < c->tune.steps_per_launch; ++k)
        if ((rc = enqueue_block_step(c, c->stream))) return rc;
    }
    if ((rc = readback(c))) return rc;
    if (*(const int32_t *)(c->pinned + 16)) break;
    if (c->pinned[nbk::kCtrNotDone] == 0) break;
    if (++launches > max_launches) return fail(NBODY_EHIP, "block steps did not reach t_end");
  }
  if ((rc = take_error(c))) return rc;
  for (int k = 0; k < c->C; ++k) c->T_host[k] = tend;
  if (n_block_steps) *n_block_steps = c->pinned[nbk::kCtrSteps] - steps0;
  if (n_interactions) *n_interactions = c->pinned[nbk::kCtrInter] - inter0;
  return NBODY_OK;
}

int nbody_step_blocks(nbody_ctx *c, double t_end, int64_t max_block_steps,
                      int64_t *n_block_steps, int64_t *n_interactions) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  if (max_block_steps < 0) return fail(NBODY_EINVAL, "max_block_steps < 0");
  int64_t tend = 0;
  int rc = check_t_end(c, t_end, &tend);
  if (rc) return rc;
  if ((rc = readback(c))) return rc;
  if ((rc = take_error(c))) return rc;
  const int64_t steps0 = c->pinned[nbk::kCtrSteps], inter0 = c->pinned[nbk::kCtrInter];
  NB_HIP(nbk::launch_set_word64(c->d.ctr + nbk::kCtrTend, tend, c->stream));
  for (int64_t k = 0; k < max_block_steps; ++k) {
    if ((k & 63) == 0 && c->prec == NBODY_MIXED) NB_HIP(nbk::launch_vref(c->d, nullptr, c->stream));
    if ((rc = enqueue_block_step(c, c->stream))) return rc;
    if ((k & 63) == 63 || k + 1 == max_block_steps) {
      if ((rc = readback(c))) return rc;
      if (*(const int32_t *)(c->pinned + 16)) break;
      if (c->pinned[nbk::kCtrNotDone] == 0) break;
    }
  }
  if ((rc = readback(c))) return rc;
  if ((rc = take_error(c))) return rc;
  // clusters may stop anywhere on the way: take their times from the device
  NB_HIP(hipMemcpyAsync(c->T_host.data(), c->d.T, sizeof(int64_t) * c->C,
                        hipMemcpyDeviceToHost, c->stream));
  NB_HIP(hipStreamSynchronize(c->stream));
  if (n_block_steps) *n_block_steps = c->pinned[nbk::kCtrSteps] - steps0;
  if (n_interactions) *n_interactions = c->pinned[nbk::kCtrInter] - inter0;
  return NBODY_OK;
}

int nbody_energy(nbody_ctx *c, double *out) {
  if (!c || !out) return fail(NBODY_EINVAL, "NULL argument");
  nbk::Tuning t = device_tuning(c, 1);
  // the energy sums run one workgroup per cluster, each particle's split
  // rows in turn: keep the potential evaluation to at most four j-splits
  // per i-tile (target <= 4 x the fewest i-tiles of the bucket)
  for (int b = 0; b < nbk::kBuckets; ++b) {
    int P = t.i_slots[b] < 1 ? 1 : (t.i_slots[b] > 256 ? 256 : t.i_slots[b]);
    while (P & (P - 1)) P &= P - 1;
    const int64_t tiles_min = (((int64_t)1 << b) + P - 1) / P;
    const int64_t cap = 4 * tiles_min;
    if (t.target_items[b] > cap) t.target_items[b] = (int32_t)cap;
  }
  NB_HIP(nbk::launch_all_active(c->d, t, c->stream));
  if (c->C > 1) NB_HIP(nbk::launch_plan(c->d, t, nbk::kPlanState, 0, false, c->stream));
  int rc0 = force_launch(c, nbk::kModePot, nbk::kSrcState, 1, nullptr, c->d.active, c->grid_pot,
                         c->stream);
  if (rc0) return rc0;
  NB_HIP(nbk::launch_energy_reduce(c->d, c->stream));
  NB_HIP(hipMemcpyAsync(out, c->d.eout, sizeof(double) * 9 * c->C, hipMemcpyDeviceToHost,
                        c->stream));
  int rc = readback(c);
  if (rc) return rc;
  return take_error(c);
}

int nbody_get_state(nbody_ctx *c, double *x, double *v, double *a, double *jerk,
                    int64_t *tick, int8_t *level) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  NB_HIP(nbk::launch_get_state(c->d, x, v, a, jerk, tick, level, c->stream));
  int rc = readback(c);
  if (rc) return rc;
  return take_error(c);
}

int nbody_set_state(nbody_ctx *c, const double *x, const double *v, const double *a,
                    const double *jerk, const int64_t *tick, const int8_t *level) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  if (!x || !v || !a || !jerk || !tick || !level) return fail(NBODY_EINVAL, "NULL array argument");
  int rc = readback(c);
  if (rc) return rc;
  if ((rc = take_error(c))) return rc;
  NB_HIP(nbk::launch_fill32((int32_t *)c->d.T, 0, 2 * (int64_t)c->C, c->stream));
  NB_HIP(nbk::launch_fill32(c->d.hist, 0, (int64_t)c->C * nbk::kLevels, c->stream));
  NB_HIP(nbk::launch_set_state(c->d, x, v, a, jerk, tick, level, c->lmin, c->lmax, c->stream));
  NB_HIP(hipMemcpyAsync(c->T_host.data(), c->d.T, sizeof(int64_t) * c->C, hipMemcpyDeviceToHost,
                        c->stream));
  if ((rc = readback(c))) return rc;
  return take_error(c);
}

int nbody_sync(nbody_ctx *c) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  int rc = readback(c);
  if (rc) return rc;
  return take_error(c);
}

int nbody_stats(nbody_ctx *c, int64_t *out8) {
  if (!c || !out8) return fail(NBODY_EINVAL, "NULL argument");
  int rc = readback(c);
  if (rc) return rc;
  out8[0] = c->pinned[nbk::kCtrSteps];
  out8[1] = c->pinned[nbk::kCtrInter];
  out8[2] = c->pinned[nbk::kCtrFloor];
  out8[3] = c->T_host[0];
  out8[4] = c->pinned[nbk::kCtrRefined];
  out8[5] = c->pinned[nbk::kCtrNear];
  out8[6] = c->pinned[nbk::kCtrSmallInter];
  out8[7] = 0;
  return NBODY_OK;
}

void nbody_destroy(nbody_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->pinned) (void)hipHostFree(c->pinned);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

int nbody_profile(nbody_ctx *c, int enable) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  if (enable && c->ev.empty()) {
    c->ev.assign(2 * kEvPairs, nullptr);
    c->ev_tag.assign(kEvPairs, 0);
    for (auto &e : c->ev) NB_HIP(hipEventCreate(&e));
  }
  if (!enable && c->profiling) {
    int rc = harvest_events(c);
    if (rc) return rc;
  }
  c->profiling = enable != 0;
  return NBODY_OK;
}

int nbody_profile_read(nbody_ctx *c, double *force_ms, int64_t *force_launches,
                       double *refine_ms, int64_t *refine_launches) {
  if (!c) return fail(NBODY_EINVAL, "context is NULL");
  int rc = harvest_events(c);
  if (rc) return rc;
  if (force_ms) *force_ms = c->prof_ms[0];
  if (force_launches) *force_launches = c->prof_launches[0];
  if (refine_ms) *refine_ms = c->prof_ms[1];
  if (refine_launches) *refine_launches = c->prof_launches[1];
  c->prof_ms[0] = c->prof_ms[1] = 0.0;
  c->prof_launches[0] = c->prof_launches[1] = 0;
  return NBODY_OK;
}

const char *nbody_strerror(int code) {
  switch (code) {
    case NBODY_OK: return "success";
    case NBODY_EINVAL: return "invalid argument";
    case NBODY_ENODEV: return "no usable HIP device";
    case NBODY_ENOMEM: return "workspace too small";
    case NBODY_EHIP: return "HIP runtime error";
    case NBODY_EINDEX: return "index out of range or i_active not grouped by cluster";
    case NBODY_ENONFINITE: return "non-finite value";
    case NBODY_EDOMAIN: return "coincident particles with zero softening";
    default: return "unknown error";
  }
}

const char *nbody_last_error(void) { return g_last_error.c_str(); }

int nbody_get_tuning(const nbody_ctx *c, nbody_tuning *t) {
  if (!c || !t) return fail(NBODY_EINVAL, "NULL argument");
  *t = c->tune;
  return NBODY_OK;
}

int nbody_set_tuning(nbody_ctx *c, const nbody_tuning *t) {
  if (!c || !t) return fail(NBODY_EINVAL, "NULL argument");
  nbody_tuning n = c->tune;
  if (t->variant) {
    if (t->variant != NBODY_VARIANT_K1 && t->variant != NBODY_VARIANT_K2 &&
        t->variant != NBODY_VARIANT_S1 && t->variant != NBODY_VARIANT_S2)
      return fail(NBODY_EINVAL, "unknown variant");
    n.variant = t->variant;
  }
  if (t->acc_variant) {
    if (t->acc_variant != -1 && t->acc_variant != NBODY_VARIANT_K1 &&
        t->acc_variant != NBODY_VARIANT_K2 && t->acc_variant != NBODY_VARIANT_S1 &&
        t->acc_variant != NBODY_VARIANT_S2)
      return fail(NBODY_EINVAL, "unknown acc_variant");
    n.acc_variant = t->acc_variant == -1 ? 0 : t->acc_variant;
  }
  if (t->use_graph) {
    if (t->use_graph != NBODY_GRAPH_ON && t->use_graph != NBODY_GRAPH_OFF)
      return fail(NBODY_EINVAL, "use_graph must be NBODY_GRAPH_ON or NBODY_GRAPH_OFF");
    n.use_graph = t->use_graph;
  }
  if (t->steps_per_launch) {
    if (t->steps_per_launch < 1 || t->steps_per_launch > 1024)
      return fail(NBODY_EINVAL, "steps_per_launch must be in [1, 1024]");
    n.steps_per_launch = t->steps_per_launch;
  }
  if (t->min_split_j) {
    if (t->min_split_j < 64) return fail(NBODY_EINVAL, "min_split_j must be >= 64");
    n.min_split_j = t->min_split_j;
  }
  if (t->refine_ratio != 0.0f) {
    if (!std::isfinite(t->refine_ratio)) return fail(NBODY_EINVAL, "refine_ratio must be finite");
    n.refine_ratio = t->refine_ratio;
  }
  if (t->near_jerk != 0.0f) {
    if (!std::isfinite(t->near_jerk)) return fail(NBODY_EINVAL, "near_jerk must be finite");
    n.near_jerk = t->near_jerk;
  }
  if (t->small_log2) {
    if (t->small_log2 != -1 && (t->small_log2 < 1 || t->small_log2 > 62))
      return fail(NBODY_EINVAL, "small_log2 must be -1 or in [1, 62]");
    n.small_log2 = t->small_log2;
  }
  for (int b = 0; b < NBODY_TUNE_BUCKETS; ++b) {
    if (t->i_slots[b]) {
      const int P = t->i_slots[b];
      if (P < 1 || P > 256 || (P & (P - 1))) return fail(NBODY_EINVAL, "i_slots must be a power of two in [1, 256]");
      n.i_slots[b] = P;
    }
    if (t->target_items[b]) {
      if (t->target_items[b] < 1 || t->target_items[b] > (1 << 20))
        return fail(NBODY_EINVAL, "target_items must be in [1, 2^20]");
      n.target_items[b] = t->target_items[b];
    }
  }
  c->tune = n;
  drop_graph(c);
  return refresh_grids(c);
}

}  // extern "C"

// ---- evaluation without any allocation ------------------------------------
//
// nbody_forces_noalloc: the evaluation of nbody_forces for one cluster of at
// most kStaticMaxN particles, without a context and without any allocation.
// Its scratch (plan, partial rows, j records, near-pair queue thresholds,
// re-evaluation lists) lives in the file-scope device array `scratch`; the
// host side of the evaluation is a per-device static context that only ever
// holds plain values.  On each device, the first call takes the array's
// device address with hipGetSymbolAddress (with that device current) and
// keeps it; kernels receive that address, never the array's name.

namespace {

constexpr int64_t kStaticMaxN = 16384;        // particles (n_j and n_active)
constexpr int kStaticRowsPerJ = 4;            // partial rows per j-particle
constexpr size_t kStaticBytes = (size_t)16 << 20;
constexpr int kStaticDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

struct StaticCtx {
  bool ready = false;
  char *base = nullptr;       // device address of `scratch` on this device
  int grids_prec = -1;        // precision the launch grids were sized for
  nbody_ctx ctx;              // empty vectors only: nothing is allocated
};

StaticCtx g_static[kStaticDevices];
std::mutex g_static_mu;

}  // namespace

extern "C" {

int nbody_forces_noalloc(int precision, double eps, const int32_t *i_active, int64_t n_active,
                         const double *xj, const double *vj, const double *mj, int64_t n_j,
                         double *acc, double *jerk, void *stream) {
  if (precision != NBODY_FP64 && precision != NBODY_MIXED && precision != NBODY_MIXED_DS)
    return fail(NBODY_EINVAL, "unknown precision");
  if (!std::isfinite(eps) || eps < 0.0) return fail(NBODY_EINVAL, "eps must be finite and >= 0");
  if (n_active < 0) return fail(NBODY_EINVAL, "n_active < 0");
  if (n_j < 1 || n_j > kStaticMaxN)
    return fail(NBODY_EINVAL, "n_j must be in [1, 16384] for nbody_forces_noalloc");
  if (n_active > kStaticMaxN)
    return fail(NBODY_EINVAL, "n_active must be at most 16384 for nbody_forces_noalloc");
  if (n_active == 0) return NBODY_OK;
  if (!i_active || !xj || !vj || !mj || !acc) return fail(NBODY_EINVAL, "NULL array argument");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(NBODY_ENODEV, "no current HIP device");
  if (dev < 0 || dev >= kStaticDevices) return fail(NBODY_ENODEV, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticCtx &g = g_static[dev];
  if (!g.ready) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NBODY_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (carve(kStaticMaxN, 1, nullptr, nullptr, kStaticRowsPerJ) > kStaticBytes)
      return fail(NBODY_EHIP, "static scratch smaller than its largest evaluation");
    g.base = (char *)p;
    g.ctx.device = dev;
    g.ready = true;
  }
  nbody_ctx *c = &g.ctx;
  c->stream = (hipStream_t)stream;
  c->n = n_j;
  c->C = 1;
  carve(n_j, 1, g.base, &c->d, kStaticRowsPerJ);
  c->d.fld = nbk::Field{};
  if (g.grids_prec != precision) {
    c->prec = precision;
    c->tune = default_tuning(precision);
    int rc = refresh_grids(c);
    if (rc) return rc;
    g.grids_prec = precision;
  }
  // the cluster table of this call: [0, n_j) and eps^2 (kernels, no copies)
  const double eps2 = eps * eps;
  int64_t eps2_bits;
  std::memcpy(&eps2_bits, &eps2, sizeof eps2_bits);
  NB_HIP(nbk::launch_set_word64(c->d.coff, 0, c->stream));
  NB_HIP(nbk::launch_set_word64(c->d.coff + 1, n_j, c->stream));
  NB_HIP(nbk::launch_set_word64((int64_t *)c->d.eps2, eps2_bits, c->stream));
  return api_forces(c, false, i_active, n_active, xj, vj, mj, n_j, acc, jerk);
}

}  // extern "C"
