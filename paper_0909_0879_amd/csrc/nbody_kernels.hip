// HIP kernels of the direct N-body hot path for gfx950 (MI355X).
//
// Force law: eq. (1) of the paper (Sect. 2) with G = 1 and the Plummer
// softened pair potential phi = -m / sqrt(r^2 + eps^2) (softening, Sect. 4),
// plus the jerk (time derivative of the acceleration):
//   a_i = sum_j m_j r_ij s^-3/2,
//   j_i = sum_j m_j [v_ij s^-3/2 - 3 (r_ij . v_ij) r_ij s^-5/2],
//   r_ij = x_j - x_i, v_ij = v_j - v_i, s = |r_ij|^2 + eps^2.
// Integration: fourth-order Hermite predictor-corrector on power-of-two
// block time steps (individual time steps, Sect. 3) with Aarseth's step
// criterion.
//
// Kernel layout on CDNA4:
//  * the force kernels are persistent: each 256-thread workgroup takes the
//    work item (cluster, i-tile, j-split) of its own index, then pulls further
//    ones from an atomic counter; items are ordered largest cost first
//    (k_plan), so uneven clusters balance;
//  * i-particles sit in registers, K per thread slot; j-particles reach the
//    ALUs either through a 256-record LDS tile (k_force) — predicted while
//    being copied from the SoA state for small active sets, or copied from
//    records that k_records predicts once per evaluation for large ones —
//    or, for large evaluations with full-width i-tiles, straight from the
//    records through the scalar cache into SGPRs (k_force_sb);
//  * the mixed paths keep the state in FP64 and run r^2, rsqrt, r^-3 and the
//    jerk products in FP32: with x_j - x_i and v_j - v_i as FP64
//    subtractions rounded to FP32 (its j records reach the broadcast kernel
//    as SGPR operands, so the FP64 subtracts cost little), or with x_j - x_i
//    formed in FP32 from double-single (hi, lo) pairs as (hi_j - hi_i) +
//    (lo_j - lo_i); particles dominated by one term are re-evaluated by the
//    FP64 kernel, and mixed block steps with few active particles run in
//    FP64 outright;
//  * small active sets put several lanes on one i (P i-slots x Q j-lanes,
//    P * Q = 256) and split j over workgroups; lanes are reduced with
//    wavefront shuffles in a fixed tree and splits by k_sum_flag in a fixed
//    order, so every result is deterministic;
//  * FP64 mode accumulates each tile in FP64 and folds it into a TwoSum
//    (hi, lo) pair; mixed mode does rsqrt, r^-3 and the jerk products in
//    FP32 and folds the FP32 sums of every 64 j into an FP32 TwoSum
//    (hi, lo) pair;
//  * the same kernels in acceleration-only modes serve the paper's
//    symplectic drivers (kick / drift sweeps between evaluations);
//  * the external Galactic field (Sect. 4) is O(N) and rides in the kernels
//    that use the acceleration (corrector, initial store, symplectic kicks,
//    energy), as compile-time variants launched only when a field is set.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nbody_internal.h"

namespace nbk {

namespace {

constexpr double kTick = 1.0 / (double)(1 << kTickBits);

// ------------------------------------------------------------ helpers

__device__ __forceinline__ double rsq64(double s) {
  // hardware reciprocal square root (good to about 2^-24 on gfx950) refined
  // by one third-order Newton-Raphson step on y^-2 = s (the iteration for
  // square roots named in Sect. 3): y1 = y (1 + e/2 + 3 e^2/8), e = 1 - s y^2,
  // which leaves a relative error of order e^3, far below FP64 rounding
  const double y = __builtin_amdgcn_rsq(s);
  const double e = fma(-s, y * y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

template <class T>
__device__ __forceinline__ void two_sum_into(T &hi, T &lo, T t) {
  const T s = hi + t;
  const T bp = s - hi;
  const T err = (hi - (s - bp)) + (t - bp);
  hi = s;
  lo += err;
}

// Hermite predictor, Taylor series to the jerk term (Horner form).
__device__ __forceinline__ void predict(double x, double v, double a, double j,
                                        double dt, double &xp, double &vp) {
  xp = x + dt * (v + dt * (0.5 * a + dt * (j / 6.0)));
  vp = v + dt * (a + dt * (0.5 * j));
}

__device__ __forceinline__ void predict_state(const Dev &d, int64_t i,
                                              int64_t t_pred, double xp[3],
                                              double vp[3]) {
  const int64_t n = d.n;
  const double dt = (double)(t_pred - d.tick[i]) * kTick;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    predict(d.x[c * n + i], d.v[c * n + i], d.a[c * n + i], d.j[c * n + i], dt,
            xp[c], vp[c]);
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Deterministic 256-thread block sum of an int (wave sums, then LDS).
__device__ int block_sum_i(int v, int *sh4) {
  v = wave_sum_i(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh4[w] = v;
  __syncthreads();
  const int tot = sh4[0] + sh4[1] + sh4[2] + sh4[3];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ int find_cluster(const int64_t *coff, int C,
                                            int64_t i) {
  int lo = 0, hi = C;   // coff[lo] <= i < coff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (coff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------ LDS records

struct JRec64 {          // one j-particle for FP64 and potential modes, 64 bytes
  double x, y, z, m;
  double vx, vy, vz;
  float mf;
  int32_t idx;
};

struct JRecDS {          // one j-particle for the double-single mode, 64 bytes:
  float xh, yh, zh, m;   // position and velocity as double-single pairs (hi +
  float xl, yl, zl, pad0;  // lo = the FP64 predicted value to ~48 bits), the
  float vx, vy, vz;      // mass (in units of the cluster's reference mass)
  int32_t idx;           // in FP32
  float vlx, vly, vlz, pad1;
};

// One particle for the mixed mode with FP64 position differences, 64
// bytes: the FP64 position, the velocity relative to the cluster's
// reference velocity as a (hi, lo) FP32 pair, the mass in units of the
// reference mass.  The reference is the mass-weighted mean velocity of a
// strided sample of the cluster (k_vref: refreshed between block-step
// launches for the state, taken from a caller's arrays before an evaluation
// of them).  A j-particle enters with hi alone and an i-particle with both,
// so the FP32 velocity difference hi_j - hi_i - lo_i carries only the
// rounding of v_j - v_ref, which differs from j to j (it does not add up
// coherently over the sum); the pairs whose jerk term matters at that level
// are near pairs, taken in FP64.
struct JRecV {
  double x, y, z;
  float vx, vy, vz;        // v - v_ref rounded to FP32 (hi)
  float mf;
  int32_t idx;
  float vlx, vly, vlz;     // (v - v_ref) - hi rounded to FP32 (lo): read only
  int32_t pad[2];          // when the record is an i-particle
};
static_assert(sizeof(JRecV) == 64, "one 64-byte record");

struct I64 {             // an i-particle in registers, FP64 modes
  double x[3], v[3];
};

struct IV {              // an i-particle in registers for JRecV: FP64 position,
  double x[3];           // velocity relative to the cluster's reference as a
  float vh[3], vl[3];    // (hi, lo) FP32 pair
};

struct IDS {             // an i-particle in registers, mixed mode: position
  float xh[3], xl[3], v[3], vl[3];   // and velocity as (hi, lo) pairs
};

__device__ __forceinline__ void make_i(const double *xp, const double *vp, I64 &s) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s.x[c] = xp[c];
    s.v[c] = vp[c];
  }
}

// vref: the cluster's reference velocity (JRecV form only; the other forms
// take the velocity as it is)
__device__ __forceinline__ void make_i(const double *xp, const double *vp, I64 &s,
                                       const double *vref) {
  (void)vref;
  make_i(xp, vp, s);
}

__device__ __forceinline__ void make_i(const double *xp, const double *vp, IV &s,
                                       const double *vref) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s.x[c] = xp[c];
    const double w = vp[c] - vref[c];
    s.vh[c] = (float)w;
    s.vl[c] = (float)(w - (double)s.vh[c]);
  }
}

// hi = x rounded to FP32, lo = (x - hi) rounded to FP32 (x - hi is exact in FP64)
__device__ __forceinline__ void make_i(const double *xp, const double *vp, IDS &s) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float h = (float)xp[c];
    s.xh[c] = h;
    s.xl[c] = (float)(xp[c] - (double)h);
    s.v[c] = (float)vp[c];
    s.vl[c] = (float)(vp[c] - (double)s.v[c]);
  }
}

__device__ __forceinline__ void make_i(const double *xp, const double *vp, IDS &s,
                                       const double *vref) {
  (void)vref;
  make_i(xp, vp, s);
}

// Reference mass of a cluster's FP32 sums: the mass of the first particle of
// its j range (1 if that is zero).  The FP32 pair terms take m_j / m_ref, so
// equal masses enter them as exactly 1 and the rounding of a mass such as
// 1/N does not scale all FP32 terms against the FP64 near terms of the same
// sum; the kernels scale their sums back by m_ref in FP64.
__device__ __forceinline__ double mass_ref(double m0) { return m0 != 0.0 ? m0 : 1.0; }

// FP64 records keep m exact (FP64 and potential modes) and m / m_ref in FP32.
// vref: the cluster's reference velocity, used by the JRecV form only.
__device__ __forceinline__ void make_rec(const double *xp, const double *vp, double m,
                                         int32_t idx, JRec64 &r, double mref,
                                         const double *vref) {
  (void)vref;
  r.x = xp[0]; r.y = xp[1]; r.z = xp[2]; r.m = m;
  r.vx = vp[0]; r.vy = vp[1]; r.vz = vp[2];
  r.mf = (float)(m / mref);
  r.idx = idx;
}

__device__ __forceinline__ void make_rec(const double *xp, const double *vp, double m,
                                         int32_t idx, JRecDS &r, double mref,
                                         const double *vref) {
  (void)vref;
  IDS s;
  make_i(xp, vp, s);
  r.xh = s.xh[0]; r.yh = s.xh[1]; r.zh = s.xh[2];
  r.xl = s.xl[0]; r.yl = s.xl[1]; r.zl = s.xl[2];
  r.vx = s.v[0]; r.vy = s.v[1]; r.vz = s.v[2];
  r.vlx = s.vl[0]; r.vly = s.vl[1]; r.vlz = s.vl[2];
  r.m = (float)(m / mref);
  r.pad0 = r.pad1 = 0.0f;
  r.idx = idx;
}

__device__ __forceinline__ void make_rec(const double *xp, const double *vp, double m,
                                         int32_t idx, JRecV &r, double mref,
                                         const double *vref) {
  r.x = xp[0]; r.y = xp[1]; r.z = xp[2];
  const double w[3] = {vp[0] - vref[0], vp[1] - vref[1], vp[2] - vref[2]};
  r.vx = (float)w[0];
  r.vy = (float)w[1];
  r.vz = (float)w[2];
  r.vlx = (float)(w[0] - (double)r.vx);
  r.vly = (float)(w[1] - (double)r.vy);
  r.vlz = (float)(w[2] - (double)r.vz);
  r.mf = (float)(m / mref);
  r.idx = idx;
  r.pad[0] = r.pad[1] = 0;
}

// ------------------------------------------------------------ pair terms

template <bool MASK>
__device__ __forceinline__ void pair_fp64(const I64 &I, int iidx, const JRec64 &r,
                                          double eps2, double *t, int &dom) {
  const double dx = r.x - I.x[0], dy = r.y - I.x[1], dz = r.z - I.x[2];
  const double wx = r.vx - I.v[0], wy = r.vy - I.v[1], wz = r.vz - I.v[2];
  const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  const double rv = fma(dx, wx, fma(dy, wy, dz * wz));
  double rinv = rsq64(s);
  if (MASK) {
    if (s == 0.0) {
      rinv = 0.0;
      dom |= (r.idx != iidx);
    }
  }
  const double rinv2 = rinv * rinv;
  const double mr3 = (r.m * rinv) * rinv2;
  const double al = (3.0 * rv) * rinv2;
  t[0] = fma(mr3, dx, t[0]);
  t[1] = fma(mr3, dy, t[1]);
  t[2] = fma(mr3, dz, t[2]);
  t[3] = fma(mr3, fma(-al, dx, wx), t[3]);
  t[4] = fma(mr3, fma(-al, dy, wy), t[4]);
  t[5] = fma(mr3, fma(-al, dz, wz), t[5]);
}

// Per-i quantities the mixed paths collect for k_sum_flag: `a`, a bound on
// the largest single acceleration term, max_j m_j / s_ij (a close encounter
// or a heavy neighbour dominates the sum); `f1`, double-single form only, the
// sum over the pairs left in the FP32 sums of the jerk scale m_j s_ij^-3/2
// max_c |v_ij,c|: the far field's terms mostly share a direction (the mean
// field's tide), so a part of their rounding adds up coherently, which
// matters where the jerk is a small remainder of a far field many times
// larger.
struct Bnd {
  float a, f1;
};

// FP32 factors shared by the mixed pair terms.  The hardware rsqrt is good
// to about one FP32 ulp, and r^-2 and r^-3 would carry its error two and
// three times over; with r0 = rsqrt(s), e = 1 - s r0^2 is its residual
// (one FMA; its own rounding is of second order), and r0^2 (1 + e) is 1/s
// to about half an ulp.  1/s feeds the largest-term bound, m r^-3 and the
// jerk's 3 (r.v) / s; r^-3 = (m / s) r0 keeps r0's error only once.
struct Fac32 {
  float rinv, rinv2, mq, mr3;
};

__device__ __forceinline__ Fac32 fac32(float s, float m, float r0) {
  Fac32 f;
  const float r0sq = r0 * r0;
  const float e = fmaf(-s, r0sq, 1.0f);
  f.rinv = r0;
  f.rinv2 = fmaf(r0sq, e, r0sq);
  f.mq = m * f.rinv2;       // m / s >= |this pair's acceleration term|
  f.mr3 = f.mq * r0;
  return f;
}

// Near pairs of the mixed path.  A pair's jerk term m r^-3 (v_ij - 3 (r.v)
// r / s) carries an FP32 rounding error of a few ulp of m r^-3 |v_ij| (the
// differences, 1/s and r.v each enter 3 (r.v) r / s, whose size is up to
// 3 |v_ij|), and the jerk of most particles is dominated by a handful of
// close neighbours whose terms largely cancel; those few terms set the
// error of the sum.  A pair whose jerk scale m r^-3 max_c |v_ij,c| exceeds
// the threshold th of its i (a fraction of i's jerk) is therefore left out
// of the FP32 sums and evaluated in FP64 instead (near_fp64); with th at
// 1/8 of |jerk| that is about two pairs per particle.  th = +inf turns it
// off.  Returns the wave's lane mask of near pairs (a NaN scale counts as
// near, so a non-finite input still reaches the sums) and the m r^-3 that
// the FP32 sums take: zero in the near lanes.  The compare's lane mask
// serves both the select and the queueing (one compare per pair).
__device__ __forceinline__ uint64_t near_pair(float mr3, float wx, float wy, float wz,
                                              float th, float &mr3_fp32, float &w) {
  w = fmaxf(fmaxf(fabsf(wx), fabsf(wy)), fabsf(wz));
  constexpr int kCmpUGT = 10;      // unordered or greater than
  const uint64_t m = __builtin_amdgcn_fcmpf(mr3 * w, th, kCmpUGT);
  asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(mr3_fp32) : "v"(mr3), "s"(m));
  return m;
}

// Mixed precision: x_j - x_i and v_j - v_i from the double-single pairs,
// (hi_j - hi_i) + (lo_j - lo_i), which is the FP64 difference rounded to
// FP32 within an ulp (the hi difference is exact for close pairs);
// everything after it in FP32.
// SELF: this tile may hold the i-particle itself; its slot must not count in
// the largest-term bound (its terms are exactly zero, but m_i / eps^2 is not;
// its velocity difference is zero, so it is never a near pair).
template <bool MASK, bool SELF>
__device__ __forceinline__ uint64_t pair_mixed(const IDS &I, int iidx, const JRecDS &r,
                                           float eps2, float th, float *t, int &dom,
                                           Bnd &ba) {
  const float dx = (r.xh - I.xh[0]) + (r.xl - I.xl[0]);
  const float dy = (r.yh - I.xh[1]) + (r.yl - I.xl[1]);
  const float dz = (r.zh - I.xh[2]) + (r.zl - I.xl[2]);
  const float wx = (r.vx - I.v[0]) + (r.vlx - I.vl[0]);
  const float wy = (r.vy - I.v[1]) + (r.vly - I.vl[1]);
  const float wz = (r.vz - I.v[2]) + (r.vlz - I.vl[2]);
  const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  const float rv = fmaf(dx, wx, fmaf(dy, wy, dz * wz));
  float r0 = __builtin_amdgcn_rsqf(s);
  if (MASK) {
    if (dx == 0.0f && dy == 0.0f && dz == 0.0f) {
      r0 = 0.0f;
      dom |= (r.idx != iidx);
    }
  }
  const Fac32 f = fac32(s, r.m, r0);
  const float al = (3.0f * rv) * f.rinv2;
  ba.a = fmaxf(ba.a, (SELF && r.idx == iidx) ? 0.0f : f.mq);
  float mr3, wm;
  const uint64_t nr = near_pair(f.mr3, wx, wy, wz, th, mr3, wm);
  // double-single differences carry about twice the rounding of the FP64
  // ones: the pairs left in FP32 also count in the far-field error scale
  ba.f1 = fmaf(mr3, wm, ba.f1);
  t[0] = fmaf(mr3, dx, t[0]);
  t[1] = fmaf(mr3, dy, t[1]);
  t[2] = fmaf(mr3, dz, t[2]);
  t[3] = fmaf(mr3, fmaf(-al, dx, wx), t[3]);
  t[4] = fmaf(mr3, fmaf(-al, dy, wy), t[4]);
  t[5] = fmaf(mr3, fmaf(-al, dz, wz), t[5]);
  return nr;
}

// Acceleration only: the same operations as the two functions above up to
// the acceleration sums (so both give identical accelerations), no jerk.
template <bool MASK>
__device__ __forceinline__ void pair_fp64_acc(const I64 &I, int iidx, const JRec64 &r,
                                              double eps2, double *t, int &dom) {
  const double dx = r.x - I.x[0], dy = r.y - I.x[1], dz = r.z - I.x[2];
  const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  double rinv = rsq64(s);
  if (MASK) {
    if (s == 0.0) {
      rinv = 0.0;
      dom |= (r.idx != iidx);
    }
  }
  const double rinv2 = rinv * rinv;
  const double mr3 = (r.m * rinv) * rinv2;
  t[0] = fma(mr3, dx, t[0]);
  t[1] = fma(mr3, dy, t[1]);
  t[2] = fma(mr3, dz, t[2]);
}

template <bool MASK, bool SELF>
__device__ __forceinline__ uint64_t pair_mixed_acc(const IDS &I, int iidx, const JRecDS &r,
                                               float eps2, float th, float *t, int &dom,
                                               Bnd &ba) {
  const float dx = (r.xh - I.xh[0]) + (r.xl - I.xl[0]);
  const float dy = (r.yh - I.xh[1]) + (r.yl - I.xl[1]);
  const float dz = (r.zh - I.xh[2]) + (r.zl - I.xl[2]);
  const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  float r0 = __builtin_amdgcn_rsqf(s);
  if (MASK) {
    if (dx == 0.0f && dy == 0.0f && dz == 0.0f) {
      r0 = 0.0f;
      dom |= (r.idx != iidx);
    }
  }
  const Fac32 f = fac32(s, r.m, r0);
  ba.a = fmaxf(ba.a, (SELF && r.idx == iidx) ? 0.0f : f.mq);
  t[0] = fmaf(f.mr3, dx, t[0]);
  t[1] = fmaf(f.mr3, dy, t[1]);
  t[2] = fmaf(f.mr3, dz, t[2]);
  return 0;
}

// Mixed precision with FP64 position differences: x_j - x_i is taken in
// FP64 and rounded to FP32; v_j - v_i is (v_j - v_ref) - hi_i - lo_i in FP32
// (JRecV); everything after them is the FP32 arithmetic of pair_mixed.
// SELF: the i-particle's own slot has w = -lo_i rather than zero, so its
// terms are dropped (exactly zero in FP64).
template <bool MASK, bool SELF>
__device__ __forceinline__ uint64_t pair_mixed64(const IV &I, int iidx, const JRecV &r,
                                             float eps2, float th, float *t, int &dom,
                                             Bnd &ba) {
  const float dx = (float)(r.x - I.x[0]), dy = (float)(r.y - I.x[1]),
              dz = (float)(r.z - I.x[2]);
  const float wx = (r.vx - I.vh[0]) - I.vl[0], wy = (r.vy - I.vh[1]) - I.vl[1],
              wz = (r.vz - I.vh[2]) - I.vl[2];
  const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  const float rv = fmaf(dx, wx, fmaf(dy, wy, dz * wz));
  float r0 = __builtin_amdgcn_rsqf(s);
  if (MASK) {
    if (dx == 0.0f && dy == 0.0f && dz == 0.0f) {
      r0 = 0.0f;
      dom |= (r.idx != iidx);
    }
  }
  const Fac32 f = fac32(s, r.mf, r0);
  const float al = (3.0f * rv) * f.rinv2;
  const bool self = SELF && r.idx == iidx;
  ba.a = fmaxf(ba.a, self ? 0.0f : f.mq);
  float mr3, wm;
  const uint64_t nr = near_pair(self ? 0.0f : f.mr3, wx, wy, wz, th, mr3, wm);
  t[0] = fmaf(mr3, dx, t[0]);
  t[1] = fmaf(mr3, dy, t[1]);
  t[2] = fmaf(mr3, dz, t[2]);
  t[3] = fmaf(mr3, fmaf(-al, dx, wx), t[3]);
  t[4] = fmaf(mr3, fmaf(-al, dy, wy), t[4]);
  t[5] = fmaf(mr3, fmaf(-al, dz, wz), t[5]);
  return nr;
}

template <bool MASK, bool SELF>
__device__ __forceinline__ uint64_t pair_mixed64_acc(const IV &I, int iidx, const JRecV &r,
                                                 float eps2, float th, float *t, int &dom,
                                                 Bnd &ba) {
  const float dx = (float)(r.x - I.x[0]), dy = (float)(r.y - I.x[1]),
              dz = (float)(r.z - I.x[2]);
  const float s = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
  float r0 = __builtin_amdgcn_rsqf(s);
  if (MASK) {
    if (dx == 0.0f && dy == 0.0f && dz == 0.0f) {
      r0 = 0.0f;
      dom |= (r.idx != iidx);
    }
  }
  const Fac32 f = fac32(s, r.mf, r0);
  ba.a = fmaxf(ba.a, (SELF && r.idx == iidx) ? 0.0f : f.mq);
  t[0] = fmaf(f.mr3, dx, t[0]);
  t[1] = fmaf(f.mr3, dy, t[1]);
  t[2] = fmaf(f.mr3, dz, t[2]);
  return 0;
}

// The FP64 term of a near pair (pair_fp64's arithmetic on the FP64 predicted
// states), added to the compensated FP32 sums: each component as the FP32
// pair hi = T rounded, lo = (T - hi) rounded, hi through TwoSum into
// (shi, slo) and lo into slo.
__device__ __forceinline__ void near_add(double T, float &shi, float &slo) {
  const float h = (float)T;
  const float l = (float)(T - (double)h);
  two_sum_into(shi, slo, h);
  slo += l;
}

__device__ __forceinline__ void near_fp64(const I64 &I, const JRec64 &r, double eps2,
                                          float *shi, float *slo) {
  double tt[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int dd = 0;
  pair_fp64<false>(I, -1, r, eps2, tt, dd);   // a near pair has s > 0
#pragma unroll
  for (int c = 0; c < 6; ++c) near_add(tt[c], shi[c], slo[c]);
}

// Potential -m_j / sqrt(s) (energy diagnostics).  The i's own pair is
// skipped: by s == 0 when unsoftened (MASK, as for the forces), else by
// index in the tiles that can hold i (SELF).
template <bool MASK, bool SELF>
__device__ __forceinline__ void pair_pot(const I64 &I, int iidx, const JRec64 &r,
                                         double eps2, double *t, int &dom) {
  const double dx = r.x - I.x[0], dy = r.y - I.x[1], dz = r.z - I.x[2];
  const double s = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  double rinv = rsq64(s);
  if (MASK) {
    if (s == 0.0) {
      rinv = 0.0;
      dom |= (r.idx != iidx);
    }
  }
  if (SELF && r.idx == iidx) rinv = 0.0;
  t[0] = fma(-r.m, rinv, t[0]);
}

template <int MODE> struct Traits {          // FP64 forces
  using T = double;
  using Rec = JRec64;
  using Ist = I64;
  static constexpr int NC = 6;
  static constexpr int FOLD = kTJ;           // j per compensated fold
};
template <> struct Traits<kModeMixed> {
  using T = float;
  using Rec = JRecDS;
  using Ist = IDS;
  static constexpr int NC = 6;
  static constexpr int FOLD = 64;
};
template <> struct Traits<kModeFP64Acc> {
  using T = double;
  using Rec = JRec64;
  using Ist = I64;
  static constexpr int NC = 3;
  static constexpr int FOLD = kTJ;
};
template <> struct Traits<kModeMixedAcc> {
  using T = float;
  using Rec = JRecDS;
  using Ist = IDS;
  static constexpr int NC = 3;
  static constexpr int FOLD = 64;
};
template <> struct Traits<kModeMixed64> {
  using T = float;
  using Rec = JRecV;
  using Ist = IV;
  static constexpr int NC = 6;
  static constexpr int FOLD = 64;
};
template <> struct Traits<kModeMixed64Acc> {
  using T = float;
  using Rec = JRecV;
  using Ist = IV;
  static constexpr int NC = 3;
  static constexpr int FOLD = 64;
};
template <> struct Traits<kModePot> {
  using T = double;
  using Rec = JRec64;
  using Ist = I64;
  static constexpr int NC = 1;
  static constexpr int FOLD = kTJ;
};

template <int MODE, int K>
__device__ __forceinline__ void fold(typename Traits<MODE>::T (&t)[K][Traits<MODE>::NC],
                                     typename Traits<MODE>::T (&hi)[K][Traits<MODE>::NC],
                                     typename Traits<MODE>::T (&lo)[K][Traits<MODE>::NC]) {
  using T = typename Traits<MODE>::T;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < Traits<MODE>::NC; ++c) {
      two_sum_into(hi[k][c], lo[k][c], t[k][c]);
      t[k][c] = (T)0;
    }
}

// Modes whose FP32 pairs may hand near pairs to FP64 (acceleration and jerk).
constexpr bool mode_near(int m) { return m == kModeMixed || m == kModeMixed64; }
// Modes whose records hold velocities relative to the cluster's reference
// velocity (JRecV).
constexpr bool mode_relv(int m) { return m == kModeMixed64 || m == kModeMixed64Acc; }

// One j record against the K i-particles of a lane; nr[k] is the wave's lane
// mask of near pairs with i-particle k (left out of the FP32 sums, see
// near_pair).
template <int MODE, int K, bool MASK, bool SELF>
__device__ __forceinline__ void pair_k(const typename Traits<MODE>::Rec &r,
                                       const typename Traits<MODE>::Ist (&I)[K],
                                       const int (&iidx)[K], double eps2,
                                       const float (&th)[K],
                                       typename Traits<MODE>::T (&t)[K][Traits<MODE>::NC],
                                       int (&dom)[K], Bnd (&ba)[K], uint64_t (&nr)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    nr[k] = 0;
    if constexpr (MODE == kModeMixed)
      nr[k] = pair_mixed<MASK, SELF>(I[k], iidx[k], r, (float)eps2, th[k], t[k], dom[k], ba[k]);
    else if constexpr (MODE == kModeFP64)
      pair_fp64<MASK>(I[k], iidx[k], r, eps2, t[k], dom[k]);
    else if constexpr (MODE == kModeMixedAcc)
      pair_mixed_acc<MASK, SELF>(I[k], iidx[k], r, (float)eps2, th[k], t[k], dom[k], ba[k]);
    else if constexpr (MODE == kModeFP64Acc)
      pair_fp64_acc<MASK>(I[k], iidx[k], r, eps2, t[k], dom[k]);
    else if constexpr (MODE == kModeMixed64)
      nr[k] = pair_mixed64<MASK, SELF>(I[k], iidx[k], r, (float)eps2, th[k], t[k], dom[k], ba[k]);
    else if constexpr (MODE == kModeMixed64Acc)
      pair_mixed64_acc<MASK, SELF>(I[k], iidx[k], r, (float)eps2, th[k], t[k], dom[k], ba[k]);
    else
      pair_pot<MASK, SELF>(I[k], iidx[k], r, eps2, t[k], dom[k]);
  }
}

// Near pairs wait in a per-lane queue in LDS (the j index of each, up to
// kNearQ per i-particle and work item) and are evaluated in FP64 after the
// item's FP32 loop (near_drain), where the FP32 temporaries are dead: the
// rare FP64 work then costs the hot loop no registers.  A lane with more
// near pairs than the queue holds marks its particle for the FP64
// re-evaluation of the whole evaluation.
constexpr int kNearQ = 16;

template <int MODE, int K>
struct NearQueue {
  static constexpr bool on = mode_near(MODE);
  int32_t j[on ? K : 1][on ? kNearQ : 1][on ? kWG : 1];
};

// Queue the near pairs of a group of U records (record u has index j[u]):
// the compares' lane masks, and a single wave-uniform branch per group, so
// the FP32 path stays free of branches.
template <int MODE, int K, int U>
__device__ __forceinline__ void near_push(const uint64_t (&m)[U][K], const int (&j)[U],
                                          int (&cnt)[K], NearQueue<MODE, K> &q) {
  if constexpr (mode_near(MODE)) {
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) any |= m[u][k];
    if (any) {
      const uint64_t me = 1ull << __lane_id();
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (m[u][k] & me) {
            if (cnt[k] < kNearQ) q.j[k][cnt[k]][threadIdx.x] = j[u];
            ++cnt[k];
          }
        }
    }
  }
}

// One LDS tile against K i-particles, folding the running tile sums into the
// compensated (hi, lo) pairs every FOLD records.  WIDE: every lane owns its
// i (Q = 1); otherwise lane q of a slot takes records q, q + Q, ... and
// folds once per tile.  Near pairs go to (hi, lo) as they come, so the
// sequence of operations on (hi, lo) is the same as in the broadcast kernel.
template <int MODE, int K, bool WIDE, bool MASK, bool SELF>
__device__ __forceinline__ void tile_loop(
    const typename Traits<MODE>::Rec *tile, int cnt, int q, int Q,
    const typename Traits<MODE>::Ist (&I)[K], const int (&iidx)[K], double eps2,
    const float (&th)[K],
    typename Traits<MODE>::T (&t)[K][Traits<MODE>::NC],
    typename Traits<MODE>::T (&hi)[K][Traits<MODE>::NC],
    typename Traits<MODE>::T (&lo)[K][Traits<MODE>::NC], int (&dom)[K],
    Bnd (&ba)[K], int (&ncnt)[K], NearQueue<MODE, K> &nq) {
  constexpr int F = Traits<MODE>::FOLD;
  if (WIDE) {
    for (int j0 = 0; j0 < cnt; j0 += F) {
      const int j1 = (j0 + F < cnt) ? j0 + F : cnt;
      int jj = j0;
      for (; jj + 2 <= j1; jj += 2) {
        uint64_t nr[2][K];
        int ji[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          pair_k<MODE, K, MASK, SELF>(tile[jj + u], I, iidx, eps2, th, t, dom, ba, nr[u]);
          ji[u] = tile[jj + u].idx;
        }
        near_push<MODE, K, 2>(nr, ji, ncnt, nq);
      }
      if (jj < j1) {
        uint64_t nr[1][K];
        int ji[1] = {tile[jj].idx};
        pair_k<MODE, K, MASK, SELF>(tile[jj], I, iidx, eps2, th, t, dom, ba, nr[0]);
        near_push<MODE, K, 1>(nr, ji, ncnt, nq);
      }
      fold<MODE, K>(t, hi, lo);
    }
  } else {
    for (int jj = q; jj < cnt; jj += Q) {
      uint64_t nr[1][K];
      int ji[1] = {tile[jj].idx};
      pair_k<MODE, K, MASK, SELF>(tile[jj], I, iidx, eps2, th, t, dom, ba, nr[0]);
      near_push<MODE, K, 1>(nr, ji, ncnt, nq);
    }
    fold<MODE, K>(t, hi, lo);
  }
}

struct ForceArgs {
  Dev d;
  const int32_t *active;        // i list: internal active list, the caller's
                                // i_active, or the FP64 re-evaluation list
  const double *rx, *rv, *rm;   // raw source (nbody_forces)
  const int32_t *pred_on;       // the evaluation's record flag (d.pred_on)
  int role;                     // which flags this launch serves (Role)
  int near;                     // near-pair threshold source (NearSrc)
  float near_c;                 // threshold = near_c * jerk estimate
};

// Near-pair threshold of active entry k (particle i) of a mixed evaluation
// with jerk: near_c times the magnitude of i's stored jerk (block steps),
// of the entry's jerk from a first pass (d.theta, which holds near_c |jerk|
// already), or +inf (no near pairs).
__device__ __forceinline__ float near_threshold(const ForceArgs &A, int64_t k, int i) {
  if (A.near == kNearState) {
    const Dev &d = A.d;
    const double jx = d.j[i], jy = d.j[d.n + i], jz = d.j[2 * d.n + i];
    return A.near_c * (float)sqrt(jx * jx + jy * jy + jz * jz);
  }
  if (A.near == kNearList) return A.d.theta[k];
  return INFINITY;
}

// FP64 predicted state of particle p for a near pair: the caller's arrays
// (raw source) or the state predicted to the plan's time.
__device__ __forceinline__ void near_state(const ForceArgs &A, const ClusterPlan &cp, int p,
                                           bool raw, double x[3], double v[3], double &m) {
  if (raw) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = A.rx[3 * (int64_t)p + c];
      v[c] = A.rv[3 * (int64_t)p + c];
    }
    m = A.rm[p];
  } else {
    predict_state(A.d, p, cp.t_pred, x, v);
    m = A.d.m[p];
  }
}

// The FP64 terms of the queued near pairs of one work item, in queue order
// (ascending j), into the lane's compensated sums.
template <int MODE, int K>
__device__ __forceinline__ void near_drain(const ForceArgs &A, const ClusterPlan &cp, bool raw,
                                           double mref, const int (&iidx)[K], const bool (&ok)[K],
                                           const int (&ncnt)[K], const NearQueue<MODE, K> &nq,
                                           double eps2,
                                           typename Traits<MODE>::T (&hi)[K][Traits<MODE>::NC],
                                           typename Traits<MODE>::T (&lo)[K][Traits<MODE>::NC],
                                           Bnd (&ba)[K]) {
  if constexpr (mode_near(MODE)) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!ok[k] || ncnt[k] == 0) continue;
      if (ncnt[k] > kNearQ) {    // queue overflow: the whole particle in FP64
        ba[k].a = INFINITY;
        continue;
      }
      atomicAdd((unsigned long long *)&A.d.ctr[kCtrNear], (unsigned long long)ncnt[k]);
      I64 ip;
      double mi;
      near_state(A, cp, iidx[k], raw, ip.x, ip.v, mi);
      for (int u = 0; u < ncnt[k]; ++u) {
        const int j = nq.j[k][u][threadIdx.x];
        double xj[3], vj[3], mj;
        near_state(A, cp, j, raw, xj, vj, mj);
        JRec64 r;
        make_rec(xj, vj, mj / mref, j, r, 1.0, nullptr);   // in the FP32 sums' mass unit
        near_fp64(ip, r, eps2, hi[k], lo[k]);
      }
    }
  }
}

__device__ __forceinline__ void rec_to_i(const JRec64 &r, I64 &s) {
  s.x[0] = r.x; s.x[1] = r.y; s.x[2] = r.z;
  s.v[0] = r.vx; s.v[1] = r.vy; s.v[2] = r.vz;
}

__device__ __forceinline__ void rec_to_i(const JRecDS &r, IDS &s) {
  s.xh[0] = r.xh; s.xh[1] = r.yh; s.xh[2] = r.zh;
  s.xl[0] = r.xl; s.xl[1] = r.yl; s.xl[2] = r.zl;
  s.v[0] = r.vx; s.v[1] = r.vy; s.v[2] = r.vz;
  s.vl[0] = r.vlx; s.vl[1] = r.vly; s.vl[2] = r.vlz;
}

// The cluster's reference velocity of the JRecV form, as the record
// builders take it (d.vref, from k_vref); zero where no velocity is read
// (acceleration only) or the form has none.
template <int MODE>
__device__ __forceinline__ void ref_velocity(const ForceArgs &A, const ClusterPlan &cp, bool raw,
                                             double vref[3]) {
  (void)raw;
  vref[0] = vref[1] = vref[2] = 0.0;
  if constexpr (mode_relv(MODE) && !mode_acc_only(MODE)) {
#pragma unroll
    for (int c = 0; c < 3; ++c) vref[c] = A.d.vref[3 * cp.c + c];
  }
}

__device__ __forceinline__ void rec_to_i(const JRecV &r, IV &s) {
  s.x[0] = r.x; s.x[1] = r.y; s.x[2] = r.z;
  s.vh[0] = r.vx; s.vh[1] = r.vy; s.vh[2] = r.vz;
  s.vl[0] = r.vlx; s.vl[1] = r.vly; s.vl[2] = r.vlz;
}

// ------------------------------------------------------------ force kernel

// Waves per SIMD to aim for: the compiler's choice (1 = no minimum) for
// every shape of this kernel; a hint of five waves on the record-only
// double-single kernel spills its i-state since the velocity carries a low
// part.
template <int MODE, int SRC, int K> struct ForceOcc {
  static constexpr int waves = 1;
};

// Per-cluster prefix arrays (work items, row-sum waves) in LDS: with several
// clusters every work item or wave finds its cluster by a binary search,
// which in LDS costs a few LDS reads instead of a chain of dependent global
// loads.  The launch sizes the dynamic LDS to (C + 1) ints for 1 < C <= 1024
// (4 KB at most beside the kernels' own LDS); more clusters search in
// global memory.
__host__ __device__ __forceinline__ bool prefix_in_lds(int C) { return C > 1 && C <= 1024; }

__device__ __forceinline__ void prefix_to_lds(const int32_t *src, int C, int32_t *dst) {
  for (int c = threadIdx.x; c <= C; c += blockDim.x) dst[c] = src[c];
  __syncthreads();
}

// Largest c with pre[c] <= g (pre non-decreasing, pre[0] = 0 <= g).
__device__ __forceinline__ int prefix_find(const int32_t *pre, int C, int g) {
  int lo = 0, hi = C;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Dynamic LDS bytes of the kernels that use prefix_to_lds.
inline size_t prefix_lds_bytes(int C) {
  return prefix_in_lds(C) ? sizeof(int32_t) * (size_t)(C + 1) : 0;
}

template <int MODE, int SRC, int K>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(ForceOcc<MODE, SRC, K>::waves))) void k_force(ForceArgs A) {
  using Tr = Traits<MODE>;
  using T = typename Tr::T;
  using Rec = typename Tr::Rec;
  constexpr int NC = Tr::NC;
  __shared__ Rec tile[kTJ];
  __shared__ double red[kWG / 64][K][NC];
  __shared__ Bnd red_t[kWG / 64][K];
  __shared__ NearQueue<MODE, K> nq;
  __shared__ int s_g;
  const Dev &d = A.d;
  const int tid = threadIdx.x;
  // items [0, work[2]) belong to the main launches, [work[2], total) to the
  // small-step FP64 launch (clusters of a mixed block step with few active
  // particles); records built once for this evaluation (large active sets)
  // or built here while the tile is filled (small active sets, other calls)
  // SRC == kSrcRec: the caller guarantees records (flag 1 or 2) and the
  // kernel carries no prediction or raw-load code (fewer registers)
  constexpr bool REC = SRC == kSrcRec;
  int pred_flag = 0;
  int item_base = 0, n_items = d.work[2];
  int32_t *counter = d.work;
  if (A.role == kRoleMain) {
    pred_flag = *A.pred_on;
    if (pred_flag == 2) return;     // the broadcast kernel takes these items
    if (REC && pred_flag != 1) {    // no records: a launch-order bug
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(d.err, (int)kErrState);
      return;
    }
  } else if (A.role == kRoleSmall) {
    item_base = d.work[2];
    n_items = d.item_prefix[d.C];
    counter = d.work + 1;
  }
  // a launch with no items leaves before touching the shared counter (the
  // whole grid queueing on one atomic costs more than the launch itself)
  if (n_items <= item_base) return;
  extern __shared__ int32_t s_ipre[];   // item_prefix when prefix_in_lds(C)
  const bool lds_pre = prefix_in_lds(d.C);
  if (lds_pre) prefix_to_lds(d.item_prefix, d.C, s_ipre);
  const int32_t *ipre = lds_pre ? s_ipre : d.item_prefix;
  const bool use_pred = REC || pred_flag == 1;
  const Rec *pred = reinterpret_cast<const Rec *>(d.pred);
  // each workgroup's first item is item_base + its index; later ones come
  // from the shared counter, past those first gridDim.x (a launch with fewer
  // items than workgroups then touches the counter only once per busy
  // workgroup, instead of queueing the whole grid on it)
  for (int it = 0;; ++it) {
    int g = item_base + (int)blockIdx.x;
    if (it > 0) {
      if (tid == 0) s_g = item_base + (int)gridDim.x + atomicAdd(counter, 1);
      __syncthreads();
      g = s_g;
      __syncthreads();
    }
    if (g >= n_items) break;
    // item_prefix[lo] <= g < item_prefix[lo + 1]
    const int lo = (d.C > 1) ? prefix_find(ipre, d.C, g) : 0;
    const ClusterPlan cp = d.plan_lpt[lo];
    // split-major: the workgroups that run at the same time work on the
    // same j chunk, so each XCD's L2 serves the chunk to all of them
    const int t_item = g - ((d.C > 1) ? ipre[lo] : 0);
    const int split = t_item / cp.tiles;
    const int tile_i = t_item - split * cp.tiles;
    const int64_t js = cp.jb + (int64_t)split * cp.chunk;
    const int64_t je = (js + cp.chunk < cp.je) ? js + cp.chunk : cp.je;
    const int Qlog = cp.Qlog;
    const int Q = 1 << Qlog;
    const int p = tid >> Qlog;
    const int q = tid & (Q - 1);
    const double eps2 = d.eps2[cp.c];
    // FP32 sums in units of the cluster's reference mass (mixed modes)
    const double mref = !mode_mixed(MODE) ? 1.0
                        : mass_ref(SRC == kSrcRaw ? A.rm[cp.jb] : d.m[cp.jb]);
    double vref[3];
    ref_velocity<MODE>(A, cp, SRC == kSrcRaw, vref);

    typename Tr::Ist I[K];
    int iidx[K], dom[K];
    float th[K];
    bool ok[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int slot = tile_i * cp.P * K + k * cp.P + p;
      ok[k] = slot < cp.na;
      iidx[k] = ok[k] ? A.active[cp.act_off + slot] : -1;
      dom[k] = 0;
      if (SRC == kSrcRaw && ok[k] && (iidx[k] < cp.jb || iidx[k] >= cp.je)) {
        ok[k] = false;
        if (q == 0 && split == 0) atomicOr(d.err, (int)kErrIndex);
      }
      // the FP32 jerk scales are in units of mref
      th[k] = (mode_near(MODE) && ok[k])
                  ? (float)(near_threshold(A, cp.act_off + slot, iidx[k]) / mref)
                  : INFINITY;
      double xp[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};
      if (!ok[k]) {
        iidx[k] = -1;
      } else if (use_pred) {
        rec_to_i(pred[iidx[k]], I[k]);
        continue;
      } else if constexpr (SRC == kSrcState) {
        predict_state(d, iidx[k], cp.t_pred, xp, vp);
      } else if constexpr (SRC == kSrcRaw) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xp[c] = A.rx[3 * (int64_t)iidx[k] + c];
          vp[c] = mode_acc_only(MODE) ? 0.0 : A.rv[3 * (int64_t)iidx[k] + c];
        }
      }
      make_i(xp, vp, I[k], vref);
    }
    T t[K][NC], shi[K][NC], slo[K][NC];
    Bnd ba[K];
    int ncnt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ba[k].a = ba[k].f1 = 0.0f;
      ncnt[k] = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) t[k][c] = shi[k][c] = slo[k][c] = (T)0;
    }

    const bool mask = (eps2 == 0.0);
    for (int64_t jt = js; jt < je; jt += kTJ) {
      const int cnt = (int)((je - jt < kTJ) ? je - jt : kTJ);
      if (tid < cnt && use_pred) {
        tile[tid] = pred[jt + tid];
      } else if (!REC && tid < cnt) {
        const int64_t j = jt + tid;
        double xp[3], vp[3], m;
        if constexpr (SRC == kSrcState) {
          predict_state(d, j, cp.t_pred, xp, vp);
          m = d.m[j];
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            xp[c] = A.rx[3 * j + c];
            vp[c] = mode_acc_only(MODE) ? 0.0 : A.rv[3 * j + c];
          }
          m = A.rm[j];
        }
        Rec r;
        make_rec(xp, vp, m, (int32_t)j, r, mref, vref);
        tile[tid] = r;
      }
      // the tile barrier also tells whether any i of this workgroup lies in
      // the tile (a handful of tiles per item: the active list is ascending)
      int mine = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) mine |= (iidx[k] >= jt && iidx[k] < jt + cnt);
      const bool self_tile = __syncthreads_or(mine) != 0;
      // the FP64 force terms of the i's own pair are exactly zero; the
      // mixed bound and the potential must skip it
      constexpr bool has_self = mode_mixed(MODE) || MODE == kModePot;
      if (Q == 1) {
        if (mask)
          tile_loop<MODE, K, true, true, false>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
        else if (has_self && self_tile)
          tile_loop<MODE, K, true, false, true>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
        else
          tile_loop<MODE, K, true, false, false>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
      } else {
        if (mask)
          tile_loop<MODE, K, false, true, false>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
        else if (has_self && self_tile)
          tile_loop<MODE, K, false, false, true>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
        else
          tile_loop<MODE, K, false, false, false>(tile, cnt, q, Q, I, iidx, eps2, th, t, shi, slo, dom, ba, ncnt, nq);
      }
      __syncthreads();
    }

    near_drain<MODE, K>(A, cp, SRC == kSrcRaw, mref, iidx, ok, ncnt, nq, eps2, shi, slo, ba);
    // combine hi + lo in FP64, reduce the Q lanes of a slot in a fixed tree
    double res[K][NC];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int c = 0; c < NC; ++c) res[k][c] = ((double)shi[k][c] + (double)slo[k][c]) * mref;
      if (ok[k] && dom[k]) atomicOr(d.err, (int)kErrDomain);
    }
    if (Q > 1) {
      const int qw = Q < 64 ? Q : 64;
      for (int off = 1; off < qw; off <<= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
          for (int c = 0; c < NC; ++c) res[k][c] += __shfl_xor(res[k][c], off);
          ba[k].a = fmaxf(ba[k].a, __shfl_xor(ba[k].a, off));
          ba[k].f1 += __shfl_xor(ba[k].f1, off);
        }
      }
      if (Q > 64) {
        const int w = tid >> 6;
        if ((tid & 63) == 0) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < NC; ++c) red[w][k][c] = res[k][c];
            red_t[w][k] = ba[k];
          }
        }
        __syncthreads();
        if (q == 0) {
          const int nw = Q >> 6;   // waves of this slot: w .. w + nw - 1
#pragma unroll
          for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              double s = red[w][k][c];
              for (int u = 1; u < nw; ++u) s += red[w + u][k][c];
              res[k][c] = s;
            }
            Bnd tm = red_t[w][k];
            for (int u = 1; u < nw; ++u) {
              tm.a = fmaxf(tm.a, red_t[w + u][k].a);
              tm.f1 += red_t[w + u][k].f1;
            }
            ba[k] = tm;
          }
        }
        __syncthreads();
      }
    }
    if (q == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int slot = tile_i * cp.P * K + k * cp.P + p;
        if (slot < cp.na) {
          double *row = d.partial + (cp.row_off + (int64_t)split * cp.na + slot) * kRowStride;
#pragma unroll
          for (int c = 0; c < NC; ++c) row[c] = ok[k] ? res[k][c] : 0.0;
          if (MODE != kModePot) {
#pragma unroll
            for (int c = NC; c < 6; ++c) row[c] = 0.0;    // no jerk in acc-only modes
            row[6] = ok[k] ? (double)ba[k].a * mref : 0.0;
            row[7] = ok[k] ? (double)ba[k].f1 * mref : 0.0;
          }
        }
      }
    }
  }
}

// Sum the S partial rows of one active slot in split order (Neumaier).
__device__ __forceinline__ void sum_rows(const Dev &d, const ClusterPlan &cp,
                                         int slot, int nc, double *out) {
  double s[6], cc[6];
  for (int c = 0; c < nc; ++c) s[c] = cc[c] = 0.0;
  for (int sp = 0; sp < cp.S; ++sp) {
    const double *row = d.partial + (cp.row_off + (int64_t)sp * cp.na + slot) * kRowStride;
    for (int c = 0; c < nc; ++c) {
      const double x = row[c];
      const double u = s[c] + x;
      cc[c] += (fabs(s[c]) >= fabs(x)) ? (s[c] - u) + x : (x - u) + s[c];
      s[c] = u;
    }
  }
  for (int c = 0; c < nc; ++c) out[c] = s[c] + cc[c];
}

__device__ __forceinline__ bool finite3(const double *a) {
  return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]);
}

__device__ __forceinline__ double norm3(const double *a) {
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

// Aarseth's criterion sqrt(eta (|a||a2| + |j|^2) / (|j||a3| + |a2|^2)).
__device__ double aarseth_dt(const double *a, const double *j, const double *a2,
                             const double *a3, double eta) {
  const double na = norm3(a), nj = norm3(j), n2 = norm3(a2), n3 = norm3(a3);
  const double num = na * n2 + nj * nj;
  const double den = nj * n3 + n2 * n2;
  if (den == 0.0) return INFINITY;
  return sqrt(eta * num / den);
}

// Power-of-two block rule: halve until <= dt_c (floor at level_max,
// counted); double once when dt_c >= 2 dt and t is a multiple of 2 dt and
// the doubled step stays within level_min.
__device__ int next_level(int level, double dt_c, int64_t t_tick, int lmin,
                          int lmax, int &floor_hit) {
  double dt = ldexp(1.0, -level);
  if (dt_c < dt) {
    while (dt > dt_c && level < lmax) {
      ++level;
      dt *= 0.5;
    }
    floor_hit = (dt > dt_c);
    return level;
  }
  floor_hit = 0;
  if (level > lmin && dt_c >= 2.0 * dt) {
    const int64_t two = (int64_t)1 << (kTickBits - level + 1);
    if (t_tick % two == 0) --level;
  }
  return level;
}

__device__ int initial_level(const double *a, const double *j, double eta_s,
                             int lmin, int lmax, int &floor_hit) {
  const double na = norm3(a), nj = norm3(j);
  const double dt0 = (nj == 0.0) ? INFINITY : eta_s * na / nj;
  int level = lmin;
  double dt = ldexp(1.0, -level);
  while (dt > dt0 && level < lmax) {
    ++level;
    dt *= 0.5;
  }
  floor_hit = (dt > dt0);
  return level;
}

// ------------------------------------------------------------ O(N) kernels

// Each cluster's reference velocity for the JRecV records: the
// mass-weighted mean velocity of a strided sample of up to kWG of its
// particles (one block per cluster, a fixed-order tree sum, so a cluster
// gets the same value alone and in an ensemble); zero for a massless
// sample.  Any value serves as long as records and kernels of one
// evaluation share it; one near the bulk velocity keeps |v - v_ref| of
// order the dispersion.  raw.x set: from a caller's arrays (one cluster:
// its n_j particles).
__global__ __launch_bounds__(kWG) void k_vref(Dev d, RawSrc raw) {
  __shared__ double sh[4][kWG];
  const int c = blockIdx.x;
  const bool api = raw.x != nullptr;
  const int64_t b = (api && d.C == 1) ? 0 : d.coff[c];
  const int64_t nc = (api && d.C == 1 && raw.n_j > 0) ? raw.n_j : d.coff[c + 1] - b;
  const int k = threadIdx.x;
  double w[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < nc) {
    const int64_t i = b + (nc <= kWG ? k : (int64_t)k * nc / kWG);
    const double m = api ? raw.m[i] : d.m[i];
#pragma unroll
    for (int q = 0; q < 3; ++q) w[q] = m * (api ? raw.v[3 * i + q] : d.v[q * d.n + i]);
    w[3] = m;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) sh[q][k] = w[q];
  __syncthreads();
  for (int off = kWG / 2; off > 0; off >>= 1) {
    if (k < off) {
#pragma unroll
      for (int q = 0; q < 4; ++q) sh[q][k] += sh[q][k + off];
    }
    __syncthreads();
  }
  if (k < 3) d.vref[3 * c + k] = sh[3][0] > 0.0 ? sh[k][0] / sh[3][0] : 0.0;
}

__global__ void k_init_state(Dev d, const double *m, const double *x,
                             const double *v) {
  const int64_t n = d.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d.x[c * n + i] = x[3 * i + c];
      d.v[c * n + i] = v[3 * i + c];
      d.a[c * n + i] = 0.0;
      d.j[c * n + i] = 0.0;
    }
    d.m[i] = m[i];
    d.tick[i] = 0;
    d.level[i] = 0;
    d.cid[i] = find_cluster(d.coff, d.C, i);
  }
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gt < 2) d.sync[gt] = 0;
  if (gt < d.C) {
    d.T[gt] = 0;
    d.Tnext[gt] = 0;
    d.Lthr[gt] = 0;
  }
  if (gt < (int64_t)d.C * kLevels) d.hist[gt] = 0;
  if (gt < kCtrCount) d.ctr[gt] = 0;
  if (gt == 0) *d.err = 0;
}

// Launch plan of cluster c whose active entries are [act_off, act_off + na):
// i-slots per workgroup from the tuning bucket of na, j-splits from the
// target item count (bounded by the split size and the partial rows), the
// items, and whether the FP64 small-step launch takes it.  row_off is left
// to the caller.
__device__ ClusterPlan plan_cluster(const Dev &d, const Tuning &tu, int kind, int64_t api_nj,
                                    int allow_small, int c, int32_t act_off, int32_t na) {
  const bool api = (kind == kPlanApi || kind == kPlanApiRefine);
  const int K = tu.K;
  ClusterPlan p;
  p.c = c;
  p.P = 256;
  p.Qlog = 0;
  p.S = 0;
  p.na = na;
  p.act_off = act_off;
  p.tiles = 0;
  p.items = 0;
  p.row_off = 0;
  p.chunk = kTJ;
  p.small = 0;
  p.glog = 0;
  if (api && d.C == 1 && api_nj > 0) {
    p.jb = 0;
    p.je = api_nj;
  } else {
    p.jb = d.coff[c];
    p.je = d.coff[c + 1];
  }
  const int64_t nc = p.je - p.jb;
  p.t_pred = (kind == kPlanStep || kind == kPlanRefine) ? d.Tnext[c] : d.T[c];
  if (p.na > 0 && nc > 0) {
    int b = 31 - __builtin_clz((unsigned)p.na);
    if (b >= kBuckets) b = kBuckets - 1;
    int P = tu.i_slots[b];
    if (P < 1) P = 1;
    if (P > 256) P = 256;
    P = 1 << (31 - __builtin_clz((unsigned)P));      // power of two
    p.P = P;
    p.Qlog = 8 - (31 - __builtin_clz((unsigned)P));
    const int64_t ipt = (int64_t)P * K;
    const int64_t tiles = (p.na + ipt - 1) / ipt;
    int64_t target = tu.target_items[b] > 0 ? tu.target_items[b] : 1;
    int64_t S = (target + tiles - 1) / tiles;
    const int64_t mj = tu.min_split_j > 0 ? tu.min_split_j : 64;
    const int64_t s_j = (nc + mj - 1) / mj;
    if (S > s_j) S = s_j;
    // partial rows of a cluster: at most kRowsPerJ per j-particle (so an
    // ensemble needs at most kRowsPerJ n rows, and a cluster splits the same
    // way alone or in an ensemble), and never more than the workspace holds
    int64_t rowcap = (int64_t)kRowsPerJ * nc;
    if (rowcap > d.rows_cap) rowcap = d.rows_cap;
    const int64_t s_r = rowcap / p.na;
    if (S > s_r) S = s_r;
    if (S < 1) S = 1;
    int64_t chunk = (nc + S - 1) / S;
    chunk = ((chunk + kTJ - 1) / kTJ) * kTJ;
    S = (nc + chunk - 1) / chunk;
    p.S = (int32_t)S;
    p.chunk = chunk;
    p.tiles = (int32_t)tiles;
    p.items = (int32_t)(tiles * S);
    int g = 0;
    while (g < 6 && (1 << g) < S) ++g;
    p.glog = g;
    p.small = (allow_small && kind == kPlanStep && tu.small_work >= 0 &&
               (p.na <= kSmallStep || (int64_t)p.na * nc <= tu.small_work)) ? 1 : 0;
  }
  return p;
}

// Waves that sum a cluster's partial rows: groups of 2^glog lanes per entry,
// 64 >> glog entries per wave.
__device__ __forceinline__ int32_t sum_waves(const ClusterPlan &p) {
  const int32_t per = 64 >> p.glog;
  return p.na > 0 ? (p.na + per - 1) / per : 0;
}

// The whole plan of a one-cluster context, by one thread: what k_plan
// writes for C = 1 (the only cluster is first in every order).  Run by the
// compaction that produced the active count, which saves a launch.
__device__ void plan_single(const Dev &d, const Tuning &tu, int kind, int64_t api_nj,
                            int allow_small, int32_t na) {
  const ClusterPlan p = plan_cluster(d, tu, kind, api_nj, allow_small, 0, 0, na);
  d.plan_c[0] = p;
  d.plan_lpt[0] = p;
  d.item_prefix[0] = 0;
  d.item_prefix[1] = p.items;
  d.sum_prefix[0] = 0;
  d.sum_prefix[1] = sum_waves(p);
  d.work[0] = 0;
  d.work[1] = 0;
  d.work[2] = p.small ? 0 : p.items;
  if (kind == kPlanStep) {
    d.T[0] = d.Tnext[0];
    if (p.items > 0) {
      d.ctr[kCtrInter] += (int64_t)p.na * (p.je - p.jb);
      if (p.small) d.ctr[kCtrSmallInter] += (int64_t)p.na * (p.je - p.jb);
      d.ctr[kCtrSteps] += 1;
    }
    d.ctr[kCtrNotDone] = (d.Tnext[0] < d.ctr[kCtrTend]) ? 1 : 0;
  }
}

__global__ void k_all_active(Dev d, Tuning tu, int plan_kind) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n;
       i += (int64_t)gridDim.x * blockDim.x)
    d.active[i] = (int32_t)i;
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gt <= d.C) d.act_off[gt] = (int32_t)d.coff[gt];
  // one cluster: every particle is active, so the plan needs nothing more
  if (gt == 0 && plan_kind >= 0) plan_single(d, tu, plan_kind, 0, 0, (int32_t)d.n);
}

// Next block-step time and threshold level of cluster c: T_next is the next
// multiple of the finest present step after T; with power-of-two steps and
// commensurate times, the particles due at T_next are exactly those with
// level >= L = 20 - ctz(T_next).  Clusters at t_end (or after an error) get
// L = kNoActive.
__device__ __forceinline__ void cluster_threshold(const Dev &d, int c, int64_t tend, int err,
                                                  int64_t *tn_out, int *L_out) {
  const int64_t T = d.T[c];
  *tn_out = T;
  *L_out = kNoActive;
  if (T >= tend || err != 0) return;
  int lmax = -1;
  for (int l = kLevels - 1; l >= 0; --l)
    if (d.hist[c * kLevels + l] > 0) { lmax = l; break; }
  if (lmax < 0) return;
  const int64_t dtl = (int64_t)1 << (kTickBits - lmax);
  const int64_t tn = (T / dtl + 1) * dtl;
  int L = kTickBits - __builtin_ctzll((unsigned long long)tn);
  if (L < 0) L = 0;
  *tn_out = tn;
  *L_out = L;
}

// Scheduler and count in one pass: each block of kScanBlock particles
// computes the threshold of the (at most kScanBlock) clusters its particles
// belong to, the block holding a cluster's first particle publishes that
// cluster's T_next and threshold, and the block counts its due particles.
__global__ __launch_bounds__(kWG) void k_count(Dev d) {
  __shared__ int sh[4];
  __shared__ int thr[kScanBlock];
  const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
  const int64_t b1 = (b0 + kScanBlock < d.n) ? b0 + kScanBlock : d.n;
  const int c0 = d.cid[b0], c1 = d.cid[b1 - 1];
  const int64_t tend = d.ctr[kCtrTend];
  const int err = *d.err;
  for (int c = c0 + threadIdx.x; c <= c1; c += kWG) {
    int64_t tn;
    int L;
    cluster_threshold(d, c, tend, err, &tn, &L);
    thr[c - c0] = L;
    const int64_t first = d.coff[c];
    if (first >= b0 && first < b1) {
      d.Tnext[c] = tn;
      d.Lthr[c] = L;
    }
  }
  __syncthreads();
  const int64_t base = b0 + threadIdx.x * 4;
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + e;
    if (i < d.n && d.level[i] >= thr[d.cid[i] - c0]) ++cnt;
  }
  cnt = block_sum_i(cnt, sh);
  if (threadIdx.x == 0) {
    d.blk_cnt[blockIdx.x] = cnt;
    d.flag_cnt[blockIdx.x] = 0;     // this step's flagging pass counts from zero
  }
}

// Sum of cnt[0, b) by the whole block (grids of at most kFusedScan blocks,
// where every block reading the counts beats a separate scan launch).
__device__ __forceinline__ int block_prefix(const int32_t *cnt, int b, int *sh4) {
  int v = 0;
  for (int u = threadIdx.x; u < b; u += kWG) v += cnt[u];
  return block_sum_i(v, sh4);
}

// Exclusive scan of nblk block counts (cnt: blk_cnt or flag_cnt) into blk_off
// by one 1024-thread workgroup.
__global__ __launch_bounds__(1024) void k_scan(Dev d, const int32_t *cnt) {
  __shared__ int sh[1024];
  int carry = 0;
  for (int base = 0; base < d.nblk; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = (i < d.nblk) ? cnt[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int add = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < d.nblk) d.blk_off[i] = carry + sh[threadIdx.x] - v;
    carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.blk_off[d.nblk] = carry;
}

// Ordered compaction: active list ascending in particle index, and each
// cluster's offset in it.  FUSED: the block sums the counts before it
// itself (no k_scan).  RMODE >= 0 (one cluster, FUSED, block steps):
// each block also writes the j records of its particles, predicted to
// T_next, in place of the record kernel (there one more launch costs more
// than the prediction), and the plan's thread sets the record flag as the
// record kernel would (0: not built; 1: built; 2: built and the broadcast
// kernel takes them, when allow_sb and the cluster's main items have kWG
// i-slots; with sb_only a flag other than 2 is reported as kErrState).
template <bool FUSED, int RMODE>
__global__ __launch_bounds__(kWG) void k_scatter(Dev d, Tuning tu, int plan_kind,
                                                 int allow_small, int allow_sb, int sb_only) {
  __shared__ int wsum[4];
  __shared__ int sh4[4];
  const int bpre = FUSED ? block_prefix(d.blk_cnt, blockIdx.x, sh4) : d.blk_off[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int flag[4];
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + e;
    flag[e] = (i < d.n && d.level[i] >= d.Lthr[d.cid[i]]) ? 1 : 0;
    cnt += flag[e];
  }
  // exclusive scan of cnt over the block, in thread order
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int wbase = 0;
  for (int u = 0; u < w; ++u) wbase += wsum[u];
  int pos = bpre + wbase + incl - cnt;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = base + e;
    if (i < d.n) {
      const int c = d.cid[i];
      if (d.coff[c] == i) d.act_off[c] = pos;
      if (flag[e]) d.active[pos++] = (int32_t)i;
    }
  }
  bool rec_on = false;
  if constexpr (RMODE >= 0) {
    // the due count of the whole cluster, for the plan's small-step test
    // (a step the FP64 small-step launch takes reads no records)
    __shared__ int sh4t[4];
    int v = 0;
    for (int u = threadIdx.x; u < d.nblk; u += kWG) v += d.blk_cnt[u];
    const int na = block_sum_i(v, sh4t);
    const bool small = allow_small && tu.small_work >= 0 &&
                       (na <= kSmallStep || (int64_t)na * d.n <= tu.small_work);
    // as the record kernel decides: mixed steps always read records, FP64
    // steps only when at least one particle in 16 is due
    rec_on = mode_mixed(RMODE) || (int64_t)na * 16 >= d.n;
    if (d.Lthr[0] != kNoActive && rec_on && !small) {
      using Rec = typename Traits<RMODE>::Rec;
      Rec *pred = reinterpret_cast<Rec *>(d.pred);
      const double mref = mode_mixed(RMODE) ? mass_ref(d.m[0]) : 1.0;
      const int64_t t1 = d.Tnext[0];
      double vref[3] = {0.0, 0.0, 0.0};     // the cluster's reference
      if constexpr (mode_relv(RMODE)) {      // velocity (JRecV form)
#pragma unroll
        for (int c = 0; c < 3; ++c) vref[c] = d.vref[c];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = (int64_t)blockIdx.x * kScanBlock + e * kWG + threadIdx.x;
        if (i < d.n) {
          double xp[3], vp[3];
          predict_state(d, i, t1, xp, vp);
          Rec r;
          make_rec(xp, vp, d.m[i], (int32_t)i, r, mref, vref);
          pred[i] = r;
        }
      }
    }
  }
  if (FUSED) {
    if (blockIdx.x == d.nblk - 1 && threadIdx.x == kWG - 1) {
      d.act_off[d.C] = pos;
      // one cluster: the active count is known here, so plan here
      if (plan_kind >= 0) plan_single(d, tu, plan_kind, 0, allow_small, pos);
      if constexpr (RMODE >= 0) {
        const ClusterPlan &p = d.plan_c[0];
        const bool elig = allow_sb && !(p.na > 0 && !p.small && p.P != kWG);
        *d.pred_on = rec_on ? (elig ? 2 : 1) : 0;
        if (sb_only && !(rec_on && elig)) atomicOr(d.err, (int)kErrState);
      }
    }
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.act_off[d.C] = d.blk_off[d.nblk];
  }
}

// Exclusive scan of one int64 per thread over a workgroup of NW waves
// (wave shuffles, then the NW wave totals); returns the prefix and sets
// *total.  sh: NW int64 of LDS.
template <int NW>
__device__ __forceinline__ int64_t block_exscan64(int64_t v, int64_t *sh, int64_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int u = 0; u < NW; ++u) {
    const int64_t t = sh[u];
    before += (u < w) ? t : 0;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Neumaier accumulation, used for the fixed-order sums over split rows.
__device__ __forceinline__ void neu_add(double &s, double &c, double x) {
  const double u = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - u) + x : (x - u) + s;
  s = u;
}

// Sum the S partial rows of one slot with a group of G = 2^glog lanes (an
// aligned part of the wave; every lane of the wave calls this, lanes of an
// idle group with valid = false): lane l of the group takes rows l, l + G,
// ... in split order, then the group combines them.  Returns the 6 sums,
// the max of column 6 and the sum of column 7, complete in the group's
// first lane (the combining rounds skip lanes that hold no row).
__device__ __forceinline__ void group_sum_rows(const Dev &d, const ClusterPlan &cp, int slot,
                                               int glog, bool valid, double *out, double &tmax,
                                               double &tf1) {
  const int G = 1 << glog;
  const int lig = threadIdx.x & (G - 1);
  double s[6], c[6];
  double tm = 0.0, f1 = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) s[q] = c[q] = 0.0;
  if (valid) {
    const double *row = d.partial + (cp.row_off + (int64_t)lig * cp.na + slot) * kRowStride;
    const int64_t step = (int64_t)G * cp.na * kRowStride;
    int sp = lig;
    // four rows in flight per lane, added in split order
    for (; sp + 3 * G < cp.S; sp += 4 * G, row += 4 * step) {
      double r[4][8];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) r[u][q] = row[u * step + q];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int q = 0; q < 6; ++q) neu_add(s[q], c[q], r[u][q]);
        tm = fmax(tm, r[u][6]);
        f1 += r[u][7];
      }
    }
    for (; sp < cp.S; sp += G, row += step) {
#pragma unroll
      for (int q = 0; q < 6; ++q) neu_add(s[q], c[q], row[q]);
      tm = fmax(tm, row[6]);
      f1 += row[7];
    }
  }
  // lanes >= S hold exact zeros, so the butterfly rounds that would only
  // add them can be skipped without changing a bit of the result
  int top = G >> 1;
  while (top > 1 && top >= cp.S) top >>= 1;
  if (!valid || cp.S <= 1) top = 0;
  // the group's shuffles stay inside the group; every lane of the wave
  // takes part in each round from the largest top in the wave down (groups
  // with a smaller top leave those rounds out)
  int start = 0;
  for (int off = 32; off >= 1; off >>= 1)
    if (__any(top >= off)) {
      start = off;
      break;
    }
  for (int off = start; off >= 1; off >>= 1) {
    const bool on = off <= top;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double os = __shfl_xor(s[q], off), oc = __shfl_xor(c[q], off);
      if (on) {
        const bool low = (threadIdx.x & off) == 0;
        const double a = low ? s[q] : os, b = low ? os : s[q];
        const double ca = low ? c[q] : oc, cb = low ? oc : c[q];
        double t = a, tc = ca + cb;
        neu_add(t, tc, b);
        s[q] = t;
        c[q] = tc;
      }
    }
    const double otm = __shfl_xor(tm, off), of1 = __shfl_xor(f1, off);
    if (on) {
      tm = fmax(tm, otm);
      // ordered by lane, so both lanes of a butterfly hold the same sum
      f1 = ((threadIdx.x & off) == 0) ? f1 + of1 : of1 + f1;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) out[q] = s[q] + c[q];
  tmax = tm;
  tf1 = f1;
}

// Cluster of active entry k: from the particle (state lists) or from the
// group offsets (caller's lists, where i indexes the caller's arrays).
__device__ __forceinline__ int entry_cluster(const Dev &d, const int32_t *list,
                                            int64_t k, bool api) {
  if (d.C == 1) return 0;
  if (!api) return d.cid[list[k]];
  int lo = 0, hi = d.C;   // largest c with act_off[c] <= k
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (d.act_off[mid] <= k) lo = mid; else hi = mid;
  }
  return lo;
}

// First slot of the re-evaluation list whose entry belongs to cluster c or a
// later one (the list of cnt slots is grouped by cluster in cluster order).
__device__ __forceinline__ int ref_list_lower(const Dev &d, int cnt, int c, bool api) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int cm = api ? entry_cluster(d, nullptr, d.ref_k[mid], true) : d.cid[d.ref_i[mid]];
    if (cm < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Launch plan for every cluster, in one workgroup of BS threads; thread t
// owns clusters t, t + BS, ..., at most QN of them (C <= BS QN), kept in
// registers.
template <int QN, int BS>
__global__ __launch_bounds__(BS) void k_plan(Dev d, Tuning tu, int kind,
                                                int64_t api_nj, int allow_small) {
  const bool refine = (kind == kPlanRefine || kind == kPlanApiRefine);
  __shared__ uint64_t key[QN * BS];           // LPT order key per cluster
  __shared__ int32_t items_by_rank[QN * BS];
  __shared__ int64_t sh[16];
  const int C = d.C;
  const int K = tu.K;
  const int tid = threadIdx.x;
  int64_t my_inter = 0, my_small = 0;
  int my_active = 0, my_notdone = 0;
  ClusterPlan cp[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int c = tid + BS * q;
    ClusterPlan &p = cp[q];
    if (c >= C) {
      p = ClusterPlan{};
      p.c = c;
      p.P = 256;
      p.chunk = kTJ;
      continue;
    }
    int32_t o0, o1;
    if (refine) {
      // re-evaluation: the cluster's range of the (cluster-grouped) flagged
      // list, whose length the ordered compaction left in blk_off[nblk]
      const int cnt = d.blk_off[d.nblk];
      o0 = ref_list_lower(d, cnt, c, kind == kPlanApiRefine);
      o1 = (c + 1 == C) ? cnt : ref_list_lower(d, cnt, c + 1, kind == kPlanApiRefine);
      d.ref_off[c] = o0;
      if (c + 1 == C) {
        d.ref_off[C] = cnt;
        d.ctr[kCtrRefined] += cnt;
      }
    } else {
      o0 = d.act_off[c];
      o1 = d.act_off[c + 1];
    }
    p = plan_cluster(d, tu, kind, api_nj, allow_small, c, o0, o1 - o0);
    if (p.items > 0) {
      my_inter += (int64_t)p.na * (p.je - p.jb);
      if (p.small) my_small += (int64_t)p.na * (p.je - p.jb);
      my_active += p.na;
    }
    if (kind == kPlanStep && d.Tnext[c] < d.ctr[kCtrTend]) ++my_notdone;
    // main-kernel clusters first, then small-step ones; within each, largest
    // item cost first, ties by cluster id (keys are unique)
    const uint64_t cost = p.items > 0 ? (uint64_t)p.P * K * p.chunk : 0;   // < 2^40
    key[c] = ((uint64_t)p.small << 63) | ((((uint64_t)1 << 40) - 1 - cost) << 12) |
             (uint64_t)c;
  }
  // partial-row offsets and row-sum waves in cluster order
  int64_t carry = 0, wcarry = 0;
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    if (BS * q >= C) break;                       // uniform
    int64_t tot;
    const int64_t r = (int64_t)cp[q].S * cp[q].na;
    cp[q].row_off = carry + block_exscan64<BS / 64>(r, sh, &tot);
    carry += tot;
    const int c = tid + BS * q;
    const int64_t wv = (c < C) ? sum_waves(cp[q]) : 0;
    const int64_t wpre = wcarry + block_exscan64<BS / 64>(wv, sh, &tot);
    if (c < C) d.sum_prefix[c] = (int32_t)wpre;
    wcarry += tot;
  }
  if (tid == 0) d.sum_prefix[C] = (int32_t)wcarry;
  __syncthreads();                                  // keys complete
  // rank of each owned cluster in LPT order
  int rank[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) rank[q] = 0;
  uint64_t mine[QN];
#pragma unroll
  for (int q = 0; q < QN; ++q) mine[q] = (tid + BS * q < C) ? key[tid + BS * q] : ~0ull;
  int u = 0;
  for (; u + 4 <= C; u += 4) {
    const uint64_t k0 = key[u], k1 = key[u + 1], k2 = key[u + 2], k3 = key[u + 3];
#pragma unroll
    for (int q = 0; q < QN; ++q)
      rank[q] += (k0 < mine[q]) + (k1 < mine[q]) + (k2 < mine[q]) + (k3 < mine[q]);
  }
  for (; u < C; ++u) {
    const uint64_t k0 = key[u];
#pragma unroll
    for (int q = 0; q < QN; ++q) rank[q] += (k0 < mine[q]);
  }
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int c = tid + BS * q;
    if (c >= C) continue;
    d.plan_c[c] = cp[q];
    d.plan_lpt[rank[q]] = cp[q];
    items_by_rank[rank[q]] = cp[q].items;
  }
  __syncthreads();
  // item prefix over the LPT order; the main items come first
  carry = 0;
  int64_t big = 0;
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    if (BS * q >= C) break;
    const int r = tid + BS * q;
    const int64_t it = (r < C) ? items_by_rank[r] : 0;
    int64_t tot;
    const int64_t pre = block_exscan64<BS / 64>(it, sh, &tot);
    if (r < C) d.item_prefix[r] = (int32_t)(carry + pre);
    carry += tot;
  }
#pragma unroll
  for (int q = 0; q < QN; ++q)
    if (tid + BS * q < C && !cp[q].small) big += cp[q].items;
  __shared__ int64_t big_sh;
  if (tid == 0) big_sh = 0;
  __syncthreads();
  if (big) atomicAdd((unsigned long long *)&big_sh, (unsigned long long)big);
  __syncthreads();
  if (tid == 0) {
    d.item_prefix[C] = (int32_t)carry;
    d.work[0] = 0;            // item counter of the main kernels
    d.work[1] = 0;            // item counter of the small-step FP64 kernel
    d.work[2] = (int32_t)big_sh;   // items [0, big) are main, [big, total) small
  }
  if (kind == kPlanStep) {
    for (int c = tid; c < C; c += BS) d.T[c] = d.Tnext[c];
    // block totals (deterministic: integer atomics)
    if (my_inter) atomicAdd((unsigned long long *)&d.ctr[kCtrInter],
                            (unsigned long long)my_inter);
    if (my_small) atomicAdd((unsigned long long *)&d.ctr[kCtrSmallInter],
                            (unsigned long long)my_small);
    __shared__ int any_active, notdone;
    if (tid == 0) { any_active = 0; notdone = 0; }
    __syncthreads();
    if (my_active) atomicAdd(&any_active, my_active);
    if (my_notdone) atomicAdd(&notdone, my_notdone);
    __syncthreads();
    if (tid == 0) {
      if (any_active) d.ctr[kCtrSteps] += 1;
      d.ctr[kCtrNotDone] = notdone;
    }
  }
}

// ------------------------------------------------------------ external field
//
// The analytic Galactic field that is added to the pairwise forces (Sect. 4):
// Plummer bulge, Miyamoto-Nagai disk, and a halo whose enclosed mass
// M(r) = hm s^(hg+1) / (1 + s^hg), s = r / ha, stops growing at hrc.  FP64,
// a few dozen operations per particle, evaluated where the integrators use
// a and jerk.  Spherical parts act as a = -G x, jerk = -(G v + H (x.v) x)
// with G = |a| / r and H = G'(r) / r; the disk term is differentiated along
// v directly.
__device__ void ext_field(const Field &f, const double x[3], const double v[3],
                          double a[3], double jk[3]) {
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const double xv = x[0] * v[0] + x[1] * v[1] + x[2] * v[2];
  double G = 0.0, H = 0.0;
  if (f.bm != 0.0) {
    const double q = 1.0 / (r2 + f.bb * f.bb);           // (r^2 + b^2)^-1
    const double gb = f.bm * q * sqrt(q);
    G += gb;
    H -= 3.0 * gb * q;
  }
  if (f.hm != 0.0 && r2 > 0.0) {
    const double r = sqrt(r2);
    double mr = f.hmc, mp = 0.0;                        // M(r), dM/dr
    if (r < f.hrc) {
      const double s = r / f.ha, sg = pow(s, f.hg), w = 1.0 / (1.0 + sg);
      mr = f.hm * s * sg * w;
      mp = (f.hm / f.ha) * sg * (f.hg + 1.0 + sg) * w * w;
    }
    const double ir3 = 1.0 / (r2 * r);
    G += mr * ir3;
    H += (mp - 3.0 * mr / r) * ir3 / r;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a[c] = -G * x[c];
    jk[c] = -(G * v[c] + H * xv * x[c]);
  }
  if (f.dm != 0.0) {
    const double z = x[2];
    const double zeta = sqrt(z * z + f.db * f.db), u = f.da + zeta;
    const double iD2 = 1.0 / (x[0] * x[0] + x[1] * x[1] + u * u);
    const double k3 = f.dm * iD2 * sqrt(iD2);           // M / D^3
    const double w = z * u / zeta;                      // z-component of grad D^2 / 2
    const double q3 = 3.0 * (x[0] * v[0] + x[1] * v[1] + w * v[2]) * iD2;
    const double dw = v[2] * (u * f.db * f.db / (zeta * zeta * zeta) + (z * z) / (zeta * zeta));
    a[0] -= k3 * x[0];
    a[1] -= k3 * x[1];
    a[2] -= k3 * w;
    jk[0] -= k3 * (v[0] - q3 * x[0]);
    jk[1] -= k3 * (v[1] - q3 * x[1]);
    jk[2] -= k3 * (dw - q3 * w);
  }
}

// Potential of the field per unit mass.
__device__ double ext_pot(const Field &f, const double x[3]) {
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  double p = 0.0;
  if (f.bm != 0.0) p -= f.bm / sqrt(r2 + f.bb * f.bb);
  if (f.dm != 0.0) {
    const double u = f.da + sqrt(x[2] * x[2] + f.db * f.db);
    p -= f.dm / sqrt(x[0] * x[0] + x[1] * x[1] + u * u);
  }
  if (f.hm != 0.0) {
    const double r = sqrt(r2);
    p += (r < f.hrc) ? f.hpc + f.hm / (f.hg * f.ha) * log1p(pow(r / f.ha, f.hg))
                     : -f.hmc / r;
  }
  return p;
}

// Hermite-4 correction of active particle i (cluster c) with its new force
// f (pair sums: a, jerk), new level, bookkeeping.
template <bool FIELD>
__device__ __forceinline__ void correct_one(const Dev &d, int64_t i, int c, double (&f)[6],
                                            double eta, double dt_shared, int lmin, int lmax) {
  const int64_t n = d.n;
  const int64_t tn = d.Tnext[c];
  const double h = (double)(tn - d.tick[i]) * kTick;
  const double h2 = h * h, h3 = h2 * h;
  double x1[3], v1[3], a2e[3], a3v[3], a1[3], j1[3], xp[3], vp[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    predict(d.x[q * n + i], d.v[q * n + i], d.a[q * n + i], d.j[q * n + i], h, xp[q], vp[q]);
  if (FIELD) {
    // the external field at the predicted position joins the pair sums
    double fa[3], fj[3];
    ext_field(d.fld, xp, vp, fa, fj);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      f[q] += fa[q];
      f[3 + q] += fj[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double a0 = d.a[q * n + i], j0 = d.j[q * n + i];
    a1[q] = f[q];
    j1[q] = f[3 + q];
    const double da = a0 - a1[q];
    const double a2 = (-6.0 * da - h * (4.0 * j0 + 2.0 * j1[q])) / h2;
    const double a3 = (12.0 * da + 6.0 * h * (j0 + j1[q])) / h3;
    x1[q] = xp[q] + a2 * (h2 * h2 / 24.0) + a3 * (h2 * h3 / 120.0);
    v1[q] = vp[q] + a2 * (h3 / 6.0) + a3 * (h2 * h2 / 24.0);
    a2e[q] = a2 + h * a3;
    a3v[q] = a3;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    d.x[q * n + i] = x1[q];
    d.v[q * n + i] = v1[q];
    d.a[q * n + i] = a1[q];
    d.j[q * n + i] = j1[q];
  }
  d.tick[i] = tn;
  if (!(finite3(x1) && finite3(v1) && finite3(a1) && finite3(j1))) {
    atomicOr(d.err, (int)kErrNonFinite);
    return;
  }
  if (dt_shared <= 0.0) {
    const int lv = d.level[i];
    const double dtc = aarseth_dt(a1, j1, a2e, a3v, eta);
    int fl = 0;
    const int nl = next_level(lv, dtc, tn, lmin, lmax, fl);
    if (fl) atomicAdd((unsigned long long *)&d.ctr[kCtrFloor], 1ull);
    if (nl != lv) {
      atomicSub(&d.hist[c * kLevels + lv], 1);
      atomicAdd(&d.hist[c * kLevels + nl], 1);
      d.level[i] = nl;
    }
  }
}

// Row sums and corrector in one pass, for block steps without a
// re-evaluation: each entry's rows are summed by a group of lanes sized to
// its split count (as in k_sum_flag), and the group's first lane corrects.
template <bool FIELD>
__global__ __launch_bounds__(kWG) void k_sum_correct(Dev d, double eta, double dt_shared,
                                                     int lmin, int lmax) {
  const int lane = threadIdx.x & 63;
  const int nw = d.sum_prefix[d.C];
  const int wave0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  extern __shared__ int32_t s_spre[];   // sum_prefix when prefix_in_lds(C)
  const bool lds_pre = prefix_in_lds(d.C);
  if (lds_pre) {
    if (wave0 - (int)(threadIdx.x >> 6) >= nw) return;   // no wave of this block has work
    prefix_to_lds(d.sum_prefix, d.C, s_spre);
  }
  const int32_t *spre = lds_pre ? s_spre : d.sum_prefix;
  for (int w = wave0; w < nw; w += nwaves) {
    // largest c with sum_prefix[c] <= w
    const int c = (d.C > 1) ? prefix_find(spre, d.C, w) : 0;
    const ClusterPlan cp = d.plan_c[c];
    const int slot = ((w - ((d.C > 1) ? spre[c] : 0)) << (6 - cp.glog)) + (lane >> cp.glog);
    const bool valid = slot < cp.na;
    double f[6], tmax, tf1;
    group_sum_rows(d, cp, slot, cp.glog, valid, f, tmax, tf1);
    if (!valid || (lane & ((1 << cp.glog) - 1)) != 0) continue;
    const int64_t k = cp.act_off + slot;
    correct_one<FIELD>(d, d.active[k], c, f, eta, dt_shared, lmin, lmax);
  }
}

// After the initial force evaluation: store a, jerk, choose levels, build
// the level histograms.
template <bool FIELD>
__global__ __launch_bounds__(kWG) void k_init_levels(Dev d, double eta_s,
                                                     double dt_shared,
                                                     int lmin, int lmax) {
  __shared__ int lh[kLevels];
  __shared__ int same;
  const int64_t n = d.n;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
  if (threadIdx.x < kLevels) lh[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    const int64_t last = (i0 + blockDim.x - 1 < n) ? i0 + blockDim.x - 1 : n - 1;
    same = (i0 < n) && d.cid[i0] == d.cid[last];
  }
  __syncthreads();
  const int64_t i = i0 + threadIdx.x;
  if (i < n) {
    const int c = d.cid[i];
    double f[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = d.fsum[6 * i + q];
    if (FIELD) {
      // every particle sits at its cluster's time: the field at the state
      double xs[3], vs[3], fa[3], fj[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xs[q] = d.x[q * n + i];
        vs[q] = d.v[q * n + i];
      }
      ext_field(d.fld, xs, vs, fa, fj);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        f[q] += fa[q];
        f[3 + q] += fj[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      d.a[q * n + i] = f[q];
      d.j[q * n + i] = f[3 + q];
    }
    int lv;
    if (!(finite3(f) && finite3(f + 3))) {
      atomicOr(d.err, (int)kErrNonFinite);
      lv = lmax;
    } else if (dt_shared > 0.0) {
      int e;
      frexp(dt_shared, &e);
      lv = 1 - e;
    } else {
      int fl = 0;
      lv = initial_level(f, f + 3, eta_s, lmin, lmax, fl);
      if (fl) atomicAdd((unsigned long long *)&d.ctr[kCtrFloor], 1ull);
    }
    d.level[i] = lv;
    if (same) atomicAdd(&lh[lv], 1);
    else atomicAdd(&d.hist[c * kLevels + lv], 1);
  }
  __syncthreads();
  if (same && threadIdx.x < kLevels && lh[threadIdx.x])
    atomicAdd(&d.hist[d.cid[i0] * kLevels + threadIdx.x], lh[threadIdx.x]);
}

// nbody_forces with several clusters: offsets of each cluster's group in
// i_active (which must be grouped by non-decreasing cluster id).
__global__ void k_api_group(Dev d, const int32_t *ia, int64_t na, Tuning tu, int64_t api_nj) {
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int C = d.C;
  // one cluster: the active count is the caller's, so plan here
  if (C == 1 && gt == 0) plan_single(d, tu, kPlanApi, api_nj, 0, (int32_t)na);
  auto key = [&](int64_t k) -> int {
    const int32_t i = ia[k];
    if (i < 0 || i >= d.n) return C;     // invalid: sorts last
    return d.cid[i];
  };
  // with one cluster the j set is the caller's (any n_j): the force kernel
  // checks i against it; with several, i must index the context's clusters
  if (C > 1) {
    for (int64_t k = gt; k < na; k += (int64_t)gridDim.x * blockDim.x) {
      const int32_t i = ia[k];
      if (i < 0 || i >= d.n) atomicOr(d.err, (int)kErrIndex);
      if (k > 0 && key(k) < key(k - 1)) atomicOr(d.err, (int)kErrIndex);
    }
  }
  if (gt <= C) {
    if (C == 1) {
      d.act_off[gt] = (gt == 0) ? 0 : (int32_t)na;
    } else {
      int64_t lo = 0, hi = na;   // first k with key(k) >= gt
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key(mid) < gt) lo = mid + 1; else hi = mid;
      }
      d.act_off[gt] = (int32_t)lo;
    }
  }
}

__global__ void k_api_finalize(Dev d, int64_t na, double *acc, double *jerk) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < na;
       k += (int64_t)gridDim.x * blockDim.x) {
    double f[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) f[q] = d.fsum[6 * k + q];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      acc[3 * k + q] = f[q];
      if (jerk) jerk[3 * k + q] = f[3 + q];
    }
    if (!(finite3(f) && finite3(f + 3))) atomicOr(d.err, (int)kErrNonFinite);
  }
}

// Build the j records of one force evaluation once, in the LDS record
// format, when its active set is large (at least 1/16 of the j particles, so
// that each j is read by many i-tiles): the tile fill of the workgroup
// kernel is then a plain copy, and the broadcast kernel reads the records
// straight into scalar registers.  Small evaluations keep the prediction
// fused into the tile fill, which reads each j once.  The decision is taken
// on the device so that captured block steps adapt to their active sets.
// *pred_on: 0 = records not built, 1 = built, 2 = built and every cluster
// with work for the main kernels runs kWG i-slots per workgroup (the
// broadcast kernel takes the evaluation; only with allow_sb).
// always: build whatever the active count (the caller launches the
// record-only kernel); particles of small-step clusters are skipped.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_records(Dev d, int kind, RawSrc raw, int allow_sb,
                                                 int always, int sb_only) {
  using Rec = typename Traits<MODE>::Rec;
  const bool api = kind == kPlanApi;
  const int64_t nj = (api && raw.n_j > 0) ? raw.n_j : d.n;
  const int64_t total = api ? raw.n_active : (int64_t)d.act_off[d.C];
  // the flag counts of this evaluation's k_sum_flag start at zero
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < d.nblk; b += gridDim.x * blockDim.x)
    d.flag_cnt[b] = 0;
  // the buffer holds d.n records
  const bool on = (always || total * 16 >= nj) && nj <= d.n;
  if (blockIdx.x == 0) {
    int elig = (on && allow_sb) ? 1 : 0;
    if (elig) {
      for (int c = threadIdx.x; c < d.C; c += blockDim.x) {
        const ClusterPlan &p = d.plan_c[c];
        if (p.na > 0 && !p.small && p.P != kWG) elig = 0;
      }
    }
    elig = __syncthreads_and(elig);
    if (threadIdx.x == 0) {
      *d.pred_on = on ? (elig ? 2 : 1) : 0;
      // the host left out the workgroup kernel's launch, which would have
      // taken the main items here: report instead of leaving them undone
      if (sb_only && !(on && elig)) atomicOr(d.err, (int)kErrState);
    }
  }
  if (!on) return;
  Rec *pred = reinterpret_cast<Rec *>(d.pred);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nj;
       i += (int64_t)gridDim.x * blockDim.x) {
    // vref: the cluster's reference velocity (JRecV form), taken as the
    // force kernels take it
    double xp[3], vp[3], m, m0, vref[3] = {0.0, 0.0, 0.0};
    if (api) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xp[c] = raw.x[3 * i + c];
        vp[c] = raw.v ? raw.v[3 * i + c] : 0.0;
      }
      m = raw.m[i];
      const int cl = d.C == 1 ? 0 : d.cid[i];
      m0 = raw.m[d.C == 1 ? 0 : d.coff[cl]];
      if constexpr (mode_relv(MODE)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) vref[c] = d.vref[3 * cl + c];
      }
    } else {
      const int c = d.cid[i];
      if (kind == kPlanStep && (d.Lthr[c] == kNoActive || d.plan_c[c].small))
        continue;                   // not stepping, or evaluated by the FP64 launch
      const int64_t t = kind == kPlanStep ? d.Tnext[c] : d.T[c];
      predict_state(d, i, t, xp, vp);
      m = d.m[i];
      m0 = d.m[d.coff[c]];
      if constexpr (mode_relv(MODE)) {
#pragma unroll
        for (int q = 0; q < 3; ++q) vref[q] = d.vref[3 * c + q];
      }
    }
    Rec r;
    make_rec(xp, vp, m, (int32_t)i, r, mode_mixed(MODE) ? mass_ref(m0) : 1.0, vref);
    pred[i] = r;
  }
}

// ------------------------------------------------------------ broadcast kernel
//
// Every lane of a wave meets the same j record at the same time, so the
// record belongs in scalar registers: it is read through the scalar cache
// (one load per wave instead of an LDS broadcast to 64 lanes) and feeds the
// vector ALU as an operand.  No LDS tile, no barrier in the j loop, and the
// vector registers hold only i-state and sums.  Each lane owns K i-particles
// (kWG i-slots per workgroup); the sums are the same operations in the same
// order as the workgroup kernel with one j-lane per slot, so both give
// bitwise-identical rows.

template <typename T>
using ScalarPtr = const __attribute__((address_space(4))) T *;

// member-wise copies (the implicit copy constructor takes a generic pointer)
__device__ __forceinline__ JRecDS load_rec(ScalarPtr<JRecDS> p) {
  JRecDS r;
  r.xh = p->xh; r.yh = p->yh; r.zh = p->zh; r.m = p->m;
  r.xl = p->xl; r.yl = p->yl; r.zl = p->zl; r.pad0 = 0.0f;
  r.vx = p->vx; r.vy = p->vy; r.vz = p->vz; r.idx = p->idx;
  r.vlx = p->vlx; r.vly = p->vly; r.vlz = p->vlz; r.pad1 = 0.0f;
  return r;
}

__device__ __forceinline__ JRec64 load_rec(ScalarPtr<JRec64> p) {
  JRec64 r;
  r.x = p->x; r.y = p->y; r.z = p->z; r.m = p->m;
  r.vx = p->vx; r.vy = p->vy; r.vz = p->vz;
  r.mf = p->mf; r.idx = p->idx;
  return r;
}

__device__ __forceinline__ JRecV load_rec(ScalarPtr<JRecV> p) {
  JRecV r;
  r.x = p->x; r.y = p->y; r.z = p->z;
  r.vx = p->vx; r.vy = p->vy; r.vz = p->vz;
  r.mf = p->mf; r.idx = p->idx;
  r.vlx = p->vlx; r.vly = p->vly; r.vlz = p->vlz;   // unread for j-particles
  r.pad[0] = r.pad[1] = 0;
  return r;
}

// Four records per group, read with as few scalar loads as possible (a
// 64-byte load is one request to the scalar cache).
typedef float f32x16 __attribute__((ext_vector_type(16)));

// one 64-byte block per record
__device__ __forceinline__ void load4(ScalarPtr<JRecDS> p, JRecDS (&r)[4]) {
  const ScalarPtr<f32x16> b = (ScalarPtr<f32x16>)p;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x16 a = b[u];
    r[u].xh = a[0]; r[u].yh = a[1]; r[u].zh = a[2]; r[u].m = a[3];
    r[u].xl = a[4]; r[u].yl = a[5]; r[u].zl = a[6]; r[u].pad0 = 0.0f;
    r[u].vx = a[8]; r[u].vy = a[9]; r[u].vz = a[10];
    r[u].idx = __float_as_int(a[11]);
    r[u].vlx = a[12]; r[u].vly = a[13]; r[u].vlz = a[14]; r[u].pad1 = 0.0f;
  }
}

__device__ __forceinline__ void load4(ScalarPtr<JRec64> p, JRec64 (&r)[4]) {
  const ScalarPtr<f32x16> b = (ScalarPtr<f32x16>)p;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x16 a = b[u];
    r[u].x = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 0, 1));
    r[u].y = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 2, 3));
    r[u].z = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 4, 5));
    r[u].m = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 6, 7));
    r[u].vx = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 8, 9));
    r[u].vy = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 10, 11));
    r[u].vz = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 12, 13));
    r[u].mf = a[14];
    r[u].idx = __float_as_int(a[15]);
  }
}

__device__ __forceinline__ void load4(ScalarPtr<JRecV> p, JRecV (&r)[4]) {
  const ScalarPtr<f32x16> b = (ScalarPtr<f32x16>)p;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x16 a = b[u];
    r[u].x = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 0, 1));
    r[u].y = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 2, 3));
    r[u].z = __builtin_bit_cast(double, __builtin_shufflevector(a, a, 4, 5));
    r[u].vx = a[6]; r[u].vy = a[7]; r[u].vz = a[8];
    r[u].mf = a[9];
    r[u].idx = __float_as_int(a[10]);
    r[u].vlx = a[11]; r[u].vly = a[12]; r[u].vlz = a[13];
    r[u].pad[0] = r[u].pad[1] = 0;
  }
}

// A chunk of records against the lane's K i-particles, four records per
// scalar load group; near pairs go to the lane's queue.
template <int MODE, int K, bool MASK, bool SELF>
__device__ __forceinline__ void sb_run(
    ScalarPtr<typename Traits<MODE>::Rec> rec, int cnt,
    const typename Traits<MODE>::Ist (&I)[K], const int (&iidx)[K], double eps2,
    const float (&th)[K], typename Traits<MODE>::T (&t)[K][Traits<MODE>::NC],
    int (&dom)[K], Bnd (&ba)[K], int (&ncnt)[K], NearQueue<MODE, K> &nq) {
  using Rec = typename Traits<MODE>::Rec;
  int jj = 0;
  if constexpr (mode_relv(MODE) && !mode_acc_only(MODE)) {
    // JRecV (11 of its 16 dwords read for a j-particle): each group's first record is loaded
    // one group early, so the group starts without waiting on the scalar
    // cache; the prefetch address stays inside the chunk
    Rec first = load_rec(rec + 0);
    for (; jj + 4 <= cnt; jj += 4) {
      Rec r[4];
      uint64_t nr[4][K];
      int ji[4];
      r[0] = first;
      r[1] = load_rec(rec + jj + 1);
      r[2] = load_rec(rec + jj + 2);
      r[3] = load_rec(rec + jj + 3);
      first = load_rec(rec + ((jj + 4 < cnt) ? jj + 4 : cnt - 1));
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pair_k<MODE, K, MASK, SELF>(r[u], I, iidx, eps2, th, t, dom, ba, nr[u]);
        ji[u] = r[u].idx;
      }
      near_push<MODE, K, 4>(nr, ji, ncnt, nq);
    }
  } else {
    for (; jj + 4 <= cnt; jj += 4) {
      Rec r[4];
      uint64_t nr[4][K];
      int ji[4];
      load4(rec + jj, r);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pair_k<MODE, K, MASK, SELF>(r[u], I, iidx, eps2, th, t, dom, ba, nr[u]);
        ji[u] = r[u].idx;
      }
      near_push<MODE, K, 4>(nr, ji, ncnt, nq);
    }
  }
  for (; jj < cnt; ++jj) {
    const Rec r = load_rec(rec + jj);
    uint64_t nr[1][K];
    int ji[1] = {r.idx};
    pair_k<MODE, K, MASK, SELF>(r, I, iidx, eps2, th, t, dom, ba, nr[0]);
    near_push<MODE, K, 1>(nr, ji, ncnt, nq);
  }
}

// The mixed broadcast kernel with one i per lane holds five waves per SIMD
// (at most 96 VGPRs); the others keep the compiler's choice.
template <int MODE, int K> struct SbOcc {
  static constexpr int waves = (mode_near(MODE) && K == 1) ? 5 : 1;
};

template <int MODE, int K>
__global__ __launch_bounds__(kWG)
__attribute__((amdgpu_waves_per_eu(SbOcc<MODE, K>::waves))) void k_force_sb(ForceArgs A) {
  using Tr = Traits<MODE>;
  using T = typename Tr::T;
  using Rec = typename Tr::Rec;
  constexpr int NC = Tr::NC;
  constexpr int F = Tr::FOLD;
  __shared__ int s_g;
  __shared__ NearQueue<MODE, K> nq;
  const Dev &d = A.d;
  if (*A.pred_on != 2) return;      // the workgroup kernel takes this evaluation
  const int tid = threadIdx.x;
  const int n_items = d.work[2];    // the main items
  if (n_items <= 0) return;
  const Rec *pred = reinterpret_cast<const Rec *>(d.pred);
  const ScalarPtr<Rec> spred = (ScalarPtr<Rec>)d.pred;
  const bool raw = A.rx != nullptr;
  extern __shared__ int32_t s_ipre[];   // item_prefix when prefix_in_lds(C)
  const bool lds_pre = prefix_in_lds(d.C);
  if (lds_pre) prefix_to_lds(d.item_prefix, d.C, s_ipre);
  const int32_t *ipre = lds_pre ? s_ipre : d.item_prefix;
  // first item by workgroup index, later ones from the counter, as in k_force
  for (int it = 0;; ++it) {
    int g = (int)blockIdx.x;
    if (it > 0) {
      if (tid == 0) s_g = (int)gridDim.x + atomicAdd(d.work, 1);
      __syncthreads();
      g = __builtin_amdgcn_readfirstlane(s_g);
      __syncthreads();
    }
    if (g >= n_items) break;
    // item_prefix[lo] <= g < item_prefix[lo + 1] (uniform: scalar from here)
    const int lo = (d.C > 1) ? __builtin_amdgcn_readfirstlane(prefix_find(ipre, d.C, g)) : 0;
    const ClusterPlan cp = d.plan_lpt[lo];
    // split-major, as in k_force
    const int t_item = g - ((d.C > 1) ? __builtin_amdgcn_readfirstlane(ipre[lo]) : 0);
    const int split = t_item / cp.tiles;
    const int tile_i = t_item - split * cp.tiles;
    const int64_t js = cp.jb + (int64_t)split * cp.chunk;
    const int64_t je = (js + cp.chunk < cp.je) ? js + cp.chunk : cp.je;
    const double eps2 = d.eps2[cp.c];
    const double mref = !mode_mixed(MODE) ? 1.0 : mass_ref(raw ? A.rm[cp.jb] : d.m[cp.jb]);
    double vref[3];
    ref_velocity<MODE>(A, cp, raw, vref);

    typename Tr::Ist I[K];
    int iidx[K], dom[K];
    float th[K];
    bool ok[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int slot = tile_i * kWG * K + k * kWG + tid;
      ok[k] = slot < cp.na;
      iidx[k] = ok[k] ? A.active[cp.act_off + slot] : -1;
      dom[k] = 0;
      if (raw && ok[k] && (iidx[k] < cp.jb || iidx[k] >= cp.je)) {
        ok[k] = false;
        if (split == 0) atomicOr(d.err, (int)kErrIndex);
      }
      // the FP32 jerk scales are in units of mref
      th[k] = (mode_near(MODE) && ok[k])
                  ? (float)(near_threshold(A, cp.act_off + slot, iidx[k]) / mref)
                  : INFINITY;
      if (ok[k]) {
        rec_to_i(pred[iidx[k]], I[k]);
      } else {
        iidx[k] = -1;
        const double z[3] = {0.0, 0.0, 0.0};
        make_i(z, z, I[k], vref);
      }
    }
    T t[K][NC], shi[K][NC], slo[K][NC];
    Bnd ba[K];
    int ncnt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ba[k].a = ba[k].f1 = 0.0f;
      ncnt[k] = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) t[k][c] = shi[k][c] = slo[k][c] = (T)0;
    }

    const bool mask = (eps2 == 0.0);
    for (int64_t jb = js; jb < je; jb += F) {
      const int cnt = (int)((je - jb < F) ? je - jb : F);
      int mine = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) mine |= (iidx[k] >= jb && iidx[k] < jb + cnt);
      const bool self = __any(mine);
      const ScalarPtr<Rec> rb = spred + jb;
      if (mask)
        sb_run<MODE, K, true, false>(rb, cnt, I, iidx, eps2, th, t, dom, ba, ncnt, nq);
      else if (mode_mixed(MODE) && self)
        sb_run<MODE, K, false, true>(rb, cnt, I, iidx, eps2, th, t, dom, ba, ncnt, nq);
      else
        sb_run<MODE, K, false, false>(rb, cnt, I, iidx, eps2, th, t, dom, ba, ncnt, nq);
      fold<MODE, K>(t, shi, slo);
    }
    near_drain<MODE, K>(A, cp, raw, mref, iidx, ok, ncnt, nq, eps2, shi, slo, ba);

#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (ok[k] && dom[k]) atomicOr(d.err, (int)kErrDomain);
      const int slot = tile_i * kWG * K + k * kWG + tid;
      if (slot < cp.na) {
        double *row = d.partial + (cp.row_off + (int64_t)split * cp.na + slot) * kRowStride;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          row[c] = ok[k] ? ((double)shi[k][c] + (double)slo[k][c]) * mref : 0.0;
#pragma unroll
        for (int c = NC; c < 6; ++c) row[c] = 0.0;
        row[6] = ok[k] ? (double)ba[k].a * mref : 0.0;
        row[7] = ok[k] ? (double)ba[k].f1 * mref : 0.0;
      }
    }
  }
}

// ------------------------------------------------------------ symplectic drivers
//
// The paper's time-symmetric integrators as kick / drift sweeps over the
// state, with the accelerations of the last evaluation in fsum (entry k =
// particle k: every particle is active).  A stage of step c = w h is
//   v += (pending + c / 2) a;  x += c v;  a = F(x);  pending = c / 2,
// so consecutive half kicks merge and each stage costs one evaluation.  The
// external field's acceleration at the current positions (those fsum was
// evaluated at) is added in the kick itself.

// Pairwise plus external acceleration of particle i at its current position.
template <bool FIELD>
__device__ __forceinline__ void sym_acc(const Dev &d, int64_t i, double acc[3]) {
  const int64_t n = d.n;
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = d.fsum[6 * i + c];
  if (FIELD) {
    double xs[3], fa[3], fj[3];
    const double zero[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) xs[c] = d.x[c * n + i];
    ext_field(d.fld, xs, zero, fa, fj);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += fa[c];
  }
}

// Kick by ck, then drift by cd.  check: every particle must sit at its
// cluster's time (no particle in the middle of a block step).
template <bool FIELD>
__global__ void k_sym_kick_drift(Dev d, double ck, double cd, int check, Tuning tu,
                                 int plan_kind) {
  const int64_t n = d.n;
  // one cluster: plan the evaluation that follows (every particle active)
  if (blockIdx.x == 0 && threadIdx.x == 0 && plan_kind >= 0)
    plan_single(d, tu, plan_kind, 0, 0, (int32_t)n);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (check && d.tick[i] != d.T[d.cid[i]]) atomicOr(d.err, kErrState);
    bool fin = true;
    double acc[3];
    sym_acc<FIELD>(d, i, acc);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v = d.v[c * n + i];
      if (ck != 0.0) v = fma(ck, acc[c], v);
      const double x = fma(cd, v, d.x[c * n + i]);
      d.v[c * n + i] = v;
      d.x[c * n + i] = x;
      fin = fin && isfinite(x) && isfinite(v);
    }
    if (!fin) atomicOr(d.err, (int)kErrNonFinite);
  }
}

template <bool FIELD>
__global__ void k_sym_kick(Dev d, double ck) {
  const int64_t n = d.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool fin = true;
    double acc[3];
    sym_acc<FIELD>(d, i, acc);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = fma(ck, acc[c], d.v[c * n + i]);
      d.v[c * n + i] = v;
      fin = fin && isfinite(v);
    }
    if (!fin) atomicOr(d.err, (int)kErrNonFinite);
  }
}

// Advance every particle's and cluster's time by dticks.
__global__ void k_sym_advance(Dev d, int64_t dticks) {
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t i = gt; i < d.n; i += (int64_t)gridDim.x * blockDim.x) d.tick[i] += dticks;
  if (gt < d.C) {
    d.T[gt] += dticks;
    d.Tnext[gt] = d.T[gt];
  }
}

// Sum the partial rows of every active entry (split order, compensated) into
// fsum.
//  * theta_out (first pass of a mixed evaluation with jerk): store the
//    near-pair threshold near_c |jerk| of each entry in d.theta for the
//    second pass; nothing is flagged.
//  * otherwise, with ratio > 0 (mixed path), flag for the FP64 re-evaluation
//    the entries whose bound on the largest single acceleration term,
//    max_j m_j / s_ij, exceeds ratio times the net acceleration (there the
//    FP32 error of that term is not small against the result), and the
//    entries whose near-pair threshold was taken from a jerk estimate (the
//    stored jerk, or the first pass) more than kNearStaleState (stored
//    jerk, whose thresholds are halved) or kNearStale times the jerk
//    found (the near pairs were then chosen too coarsely), and, in the
//    double-single form, the entries whose far-field scale (column 7)
//    exceeds kFarRatio times the jerk (a jerk that is a small remainder of a
//    far field many times larger).
// Each entry's rows are summed by a group of lanes sized to its split count
// (the plan's glog and sum_prefix); the flag counts per kScanBlock entries
// go to flag_cnt for the ordered compaction of the flagged entries
// (k_rscatter).  APPEND (one cluster): the flagged entries go to the
// re-evaluation list through one atomic counter, in whatever order they
// come (each entry's FP64 sums do not depend on its place in the list), and
// the last of the blocks that own work waves to finish publishes the count
// and writes the re-evaluation plan (plan_kind), in place of k_rscatter.
template <bool APPEND>
__global__ __launch_bounds__(kWG) void k_sum_flag(Dev d, const int32_t *list, float ratio,
                                                  float near_c, int near_src, int theta_out,
                                                  Tuning tu, int plan_kind) {
  const int lane = threadIdx.x & 63;
  const int nw = d.sum_prefix[d.C];
  const int wave0 = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  extern __shared__ int32_t s_spre[];   // sum_prefix when prefix_in_lds(C)
  const bool lds_pre = prefix_in_lds(d.C);
  if (lds_pre) {
    if (wave0 - (int)(threadIdx.x >> 6) >= nw) return;   // no wave of this block has work
    prefix_to_lds(d.sum_prefix, d.C, s_spre);
  }
  const int32_t *spre = lds_pre ? s_spre : d.sum_prefix;
  for (int w = wave0; w < nw; w += nwaves) {
    // largest c with sum_prefix[c] <= w
    const int c = (d.C > 1) ? prefix_find(spre, d.C, w) : 0;
    const ClusterPlan cp = d.plan_c[c];
    const int slot = ((w - ((d.C > 1) ? spre[c] : 0)) << (6 - cp.glog)) + (lane >> cp.glog);
    const bool valid = slot < cp.na;
    double f[6], tmax, tf1;
    group_sum_rows(d, cp, slot, cp.glog, valid, f, tmax, tf1);
    if (!valid || (lane & ((1 << cp.glog) - 1)) != 0) continue;
    // the group's first lane finishes the entry
    const int64_t k = cp.act_off + slot;
#pragma unroll
    for (int q = 0; q < 6; ++q) d.fsum[6 * k + q] = f[q];
    const double jn = sqrt(f[3] * f[3] + f[4] * f[4] + f[5] * f[5]);
    int flag = 0;
    if (theta_out) {
      d.theta[k] = near_c * (float)jn;
    } else if (ratio > 0.0f && !cp.small) {     // small-step clusters ran in FP64
      const double an = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      flag = !(tmax <= (double)ratio * an);
      double jest = -1.0;
      if (near_src == kNearState) {
        const int i = list[k];
        const double jx = d.j[i], jy = d.j[d.n + i], jz = d.j[2 * d.n + i];
        jest = sqrt(jx * jx + jy * jy + jz * jz);
      } else if (near_src == kNearList) {
        jest = (double)d.theta[k] / (double)near_c;
      }
      if (jest >= 0.0)
        flag |= !(jest <= (near_src == kNearState ? kNearStaleState : kNearStale) * jn);
      // double-single form: the far-field scale against the jerk
      if (near_src != kNearNone && tf1 > 0.0) flag |= !(tf1 <= kFarRatio * jn);
    }
    d.rflag[k] = flag;
    // per-block counts for the ordered compaction (zeroed before this
    // evaluation's force launches, by the record kernel or, for a block step,
    // by the step's k_count)
    if (flag) {
      if constexpr (APPEND) {
        const int r = atomicAdd(&d.sync[0], 1);
        d.ref_i[r] = list[k];
        d.ref_k[r] = (int32_t)k;
      } else {
        atomicAdd(&d.flag_cnt[k / kScanBlock], 1);
      }
    }
  }
  if constexpr (APPEND) {
    // the blocks that own work waves (block 0 always) take a ticket once
    // done; every count increment of a block returned before its ticket is
    // taken (the list position is used), so the last ticket's holder reads
    // the whole count
    constexpr int kWavesPerBlock = kWG / 64;
    int owners = (nw + kWavesPerBlock - 1) / kWavesPerBlock;
    if (owners > (int)gridDim.x) owners = (int)gridDim.x;
    if (owners < 1) owners = 1;
    if ((int)blockIdx.x >= owners) return;
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(&d.sync[1], 1) == owners - 1;
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
      const int total = atomicAdd(&d.sync[0], 0);
      atomicExch(&d.sync[0], 0);     // both words start at zero for the next pass
      atomicExch(&d.sync[1], 0);
      d.blk_off[d.nblk] = total;
      d.ref_off[0] = 0;
      d.ref_off[1] = total;
      d.ctr[kCtrRefined] += total;
      plan_single(d, tu, plan_kind, 0, 0, total);
    }
  }
}

// Ordered compaction of the flagged entries (blocks of kScanBlock entries,
// counted by k_sum_flag): the re-evaluation list ref_i / ref_k, grouped by
// cluster because the active list is.  FUSED: the block sums the counts before it itself, and the
// last block publishes the total (and, for one cluster, the re-evaluation
// offsets and plan).
template <bool FUSED>
__global__ __launch_bounds__(kWG) void k_rscatter(Dev d, const int32_t *list,
                                                  int64_t na_host, Tuning tu, int plan_kind,
                                                  int64_t api_nj) {
  __shared__ int wsum[4];
  __shared__ int sh4[4];
  const int bpre = FUSED ? block_prefix(d.flag_cnt, blockIdx.x, sh4) : d.blk_off[blockIdx.x];
  const int64_t total = na_host >= 0 ? na_host : d.act_off[d.C];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
  int flag[4];
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t k = base + e;
    flag[e] = (k < total && d.rflag[k]) ? 1 : 0;
    cnt += flag[e];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int wbase = 0;
  for (int u = 0; u < w; ++u) wbase += wsum[u];
  int pos = bpre + wbase + incl - cnt;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (flag[e]) {
      const int64_t k = base + e;
      d.ref_i[pos] = list[k];
      d.ref_k[pos] = (int32_t)k;
      ++pos;
    }
  }
  if (FUSED && blockIdx.x == gridDim.x - 1 && threadIdx.x == kWG - 1) {
    d.blk_off[d.nblk] = pos;          // the total, as k_scan leaves it
    if (d.C == 1) {                   // no k_plan: offsets and plan here
      d.ref_off[0] = 0;
      d.ref_off[1] = pos;
      d.ctr[kCtrRefined] += pos;
      if (plan_kind >= 0) plan_single(d, tu, plan_kind, api_nj, 0, pos);
    }
  }
}

// Write the FP64 re-evaluations over the mixed sums of their entries: one
// wave per re-evaluated entry, in blocks [0, ref_blocks).  CORR (block
// steps): that wave also corrects its particle, and blocks [ref_blocks,
// gridDim.x) correct every other active entry from fsum, one thread each —
// the whole corrector in this launch, after the FP64 pass (which predicts
// from the state) has finished.
template <bool CORR, bool FIELD>
__global__ __launch_bounds__(kWG) void k_ref_final(Dev d, int ref_blocks, CorrectSpec cs) {
  if constexpr (CORR) {
    if ((int)blockIdx.x >= ref_blocks) {
      const int na = d.act_off[d.C];
      const int stride = ((int)gridDim.x - ref_blocks) * kWG;
      for (int k = ((int)blockIdx.x - ref_blocks) * kWG + threadIdx.x; k < na; k += stride) {
        if (d.rflag[k]) continue;           // corrected by its wave below
        const int64_t i = d.active[k];
        double f[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) f[q] = d.fsum[6 * (int64_t)k + q];
        correct_one<FIELD>(d, i, d.cid[i], f, cs.eta, cs.dt_shared, cs.lmin, cs.lmax);
      }
      return;
    }
  }
  const int total = d.ref_off[d.C];
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (ref_blocks * kWG) >> 6;
  for (int r = wave; r < total; r += nwaves) {
    int c = 0;
    if (d.C > 1) {   // largest c with ref_off[c] <= r
      int lo = 0, hi = d.C;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d.ref_off[mid] <= r) lo = mid; else hi = mid;
      }
      c = lo;
    }
    const ClusterPlan cp = d.plan_c[c];
    double f[6], tmax, tf1;
    group_sum_rows(d, cp, r - cp.act_off, 6, true, f, tmax, tf1);
    if ((threadIdx.x & 63) == 0) {
      const int64_t k = d.ref_k[r];
#pragma unroll
      for (int q = 0; q < 6; ++q) d.fsum[6 * k + q] = f[q];
      if constexpr (CORR)
        correct_one<FIELD>(d, d.ref_i[r], c, f, cs.eta, cs.dt_shared, cs.lmin, cs.lmax);
    }
  }
}

// Per-cluster diagnostics: one workgroup per cluster, fixed-order sums.
template <bool FIELD>
__global__ __launch_bounds__(kWG) void k_energy_reduce(Dev d) {
  __shared__ double sh[kWG][2];
  const int c = blockIdx.x;
  const ClusterPlan cp = d.plan_c[c];
  const int64_t b = d.coff[c], e = d.coff[c + 1];
  const int64_t T = d.T[c];
  // quantities: K, W, Lx, Ly, Lz, Px, Py, Pz, external potential energy
  double s[9], cc[9];
  for (int q = 0; q < 9; ++q) s[q] = cc[q] = 0.0;
  auto add = [&](int q, double x) {
    const double u = s[q] + x;
    cc[q] += (fabs(s[q]) >= fabs(x)) ? (s[q] - u) + x : (x - u) + s[q];
    s[q] = u;
  };
  for (int64_t i = b + threadIdx.x; i < e; i += kWG) {
    double xp[3], vp[3];
    predict_state(d, i, T, xp, vp);
    const double m = d.m[i];
    double phi;
    sum_rows(d, cp, (int)(i - cp.act_off), 1, &phi);
    add(0, 0.5 * m * (vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2]));
    add(1, 0.5 * m * phi);
    add(2, m * (xp[1] * vp[2] - xp[2] * vp[1]));
    add(3, m * (xp[2] * vp[0] - xp[0] * vp[2]));
    add(4, m * (xp[0] * vp[1] - xp[1] * vp[0]));
    add(5, m * vp[0]);
    add(6, m * vp[1]);
    add(7, m * vp[2]);
    if (FIELD) add(8, m * ext_pot(d.fld, xp));
  }
  double out[9];
  for (int q = 0; q < 9; ++q) {
    sh[threadIdx.x][0] = s[q];
    sh[threadIdx.x][1] = cc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
      double S = 0.0, Cc = 0.0;
      for (int u = 0; u < kWG; ++u) {
        for (int h = 0; h < 2; ++h) {
          const double x = sh[u][h];
          const double t = S + x;
          Cc += (fabs(S) >= fabs(x)) ? (S - t) + x : (x - t) + S;
          S = t;
        }
      }
      out[q] = S + Cc;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = d.eout + 9 * (int64_t)c;
    o[0] = out[0];
    o[1] = out[1];
    o[2] = out[0] + out[1] + out[8];
    for (int q = 0; q < 6; ++q) o[3 + q] = out[2 + q];
  }
}

__global__ void k_set_word64(int64_t *p, int64_t v) { *p = v; }

__global__ void k_fill32(int32_t *p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_get_state(Dev d, double *x, double *v, double *a, double *jk,
                            int64_t *tick, int8_t *level) {
  const int64_t n = d.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (x) x[3 * i + c] = d.x[c * n + i];
      if (v) v[3 * i + c] = d.v[c * n + i];
      if (a) a[3 * i + c] = d.a[c * n + i];
      if (jk) jk[3 * i + c] = d.j[c * n + i];
    }
    if (tick) tick[i] = d.tick[i];
    if (level) level[i] = (int8_t)d.level[i];
  }
}

// set_state pass 1: copy in, validate levels, cluster time = max tick.
__global__ void k_set_state1(Dev d, const double *x, const double *v,
                             const double *a, const double *jk,
                             const int64_t *tick, const int8_t *level,
                             int lmin, int lmax) {
  const int64_t n = d.n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d.x[c * n + i] = x[3 * i + c];
      d.v[c * n + i] = v[3 * i + c];
      d.a[c * n + i] = a[3 * i + c];
      d.j[c * n + i] = jk[3 * i + c];
    }
    const int lv = level[i];
    const int64_t tk = tick[i];
    d.tick[i] = tk;
    d.level[i] = lv;
    if (lv < lmin || lv > lmax || tk < 0) {
      atomicOr(d.err, kErrState);
      continue;
    }
    const int c = d.cid[i];
    atomicMax((unsigned long long *)&d.T[c], (unsigned long long)tk);
    atomicAdd(&d.hist[c * kLevels + lv], 1);
  }
}

// set_state pass 2: tick multiple of the step and tick <= T < tick + step.
__global__ void k_set_state2(Dev d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int lv = d.level[i];
    if (lv < 0 || lv >= kLevels) continue;   // already flagged
    const int64_t dt = (int64_t)1 << (kTickBits - lv);
    const int64_t tk = d.tick[i];
    const int64_t T = d.T[d.cid[i]];
    if (tk % dt != 0 || tk > T || T >= tk + dt) atomicOr(d.err, kErrState);
  }
  const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gt < d.C) d.Tnext[gt] = d.T[gt];
}

inline int grid_for(int64_t n, int block = kWG, int cap = 4096) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <int MODE, int SRC, int K>
hipError_t launch_force_t(const ForceArgs &A, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_force<MODE, SRC, K>), dim3(grid), dim3(kWG), prefix_lds_bytes(A.d.C),
                     s, A);
  return hipGetLastError();
}

template <int MODE, int SRC, int K>
int grid_t(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void *)k_force<MODE, SRC, K>, kWG, 0) != hipSuccess)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                            device) != hipSuccess)
    cus = 256;
  if (per_cu < 1) per_cu = 1;
  return per_cu * cus;
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t launch_init_state(const Dev &d, const double *m, const double *x,
                             const double *v, hipStream_t s) {
  int64_t need = d.n;
  if (need < (int64_t)d.C * kLevels) need = (int64_t)d.C * kLevels;
  if (need < kCtrCount) need = kCtrCount;
  const int64_t blocks = (need + kWG - 1) / kWG;
  // every cluster/hist/ctr slot needs its own thread: no cap on the grid
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)blocks), dim3(kWG), 0, s, d,
                     m, x, v);
  return hipGetLastError();
}

hipError_t launch_all_active(const Dev &d, const Tuning &t, hipStream_t s) {
  int64_t need = d.n > d.C + 1 ? d.n : d.C + 1;
  hipLaunchKernelGGL(k_all_active, dim3((unsigned)((need + kWG - 1) / kWG)),
                     dim3(kWG), 0, s, d, t, d.C == 1 ? (int)kPlanState : -1);
  return hipGetLastError();
}

bool plan_fused(const Dev &d) { return d.C == 1 && d.nblk <= kFusedScan; }

hipError_t launch_compact(const Dev &d, const Tuning &t, bool allow_small, int rec_mode,
                          bool allow_sb, bool sb_only, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(d.nblk), dim3(kWG), 0, s, d);
  const int al = allow_small ? 1 : 0, sb = allow_sb ? 1 : 0, so = sb_only ? 1 : 0;
  if (d.nblk <= kFusedScan) {
    const int pk = plan_fused(d) ? (int)kPlanStep : -1;
    if (rec_mode >= 0 && !plan_fused(d))
      return hipErrorInvalidValue;
    if (rec_mode == kModeFP64)
      hipLaunchKernelGGL((k_scatter<true, kModeFP64>), dim3(d.nblk), dim3(kWG), 0, s, d, t, pk,
                         al, sb, so);
    else if (rec_mode == kModeMixed64)
      hipLaunchKernelGGL((k_scatter<true, kModeMixed64>), dim3(d.nblk), dim3(kWG), 0, s, d, t,
                         pk, al, sb, so);
    else if (rec_mode == kModeMixed)
      hipLaunchKernelGGL((k_scatter<true, kModeMixed>), dim3(d.nblk), dim3(kWG), 0, s, d, t, pk,
                         al, sb, so);
    else
      hipLaunchKernelGGL((k_scatter<true, -1>), dim3(d.nblk), dim3(kWG), 0, s, d, t, pk, al, sb,
                         so);
  } else {
    if (rec_mode >= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d, (const int32_t *)d.blk_cnt);
    hipLaunchKernelGGL((k_scatter<false, -1>), dim3(d.nblk), dim3(kWG), 0, s, d, t, -1, al, sb,
                       so);
  }
  return hipGetLastError();
}

hipError_t launch_plan(const Dev &d, const Tuning &t, int kind, int64_t api_nj,
                       bool allow_small, hipStream_t s) {
  // the smallest workgroup that gives each cluster its own thread (fewer
  // waves to synchronise in the plan's scans and barriers)
  if (d.C <= kWG)
    hipLaunchKernelGGL((k_plan<1, kWG>), dim3(1), dim3(kWG), 0, s, d, t, kind, api_nj,
                       allow_small ? 1 : 0);
  else if (d.C <= 1024)
    hipLaunchKernelGGL((k_plan<1, 1024>), dim3(1), dim3(1024), 0, s, d, t, kind, api_nj,
                       allow_small ? 1 : 0);
  else
    hipLaunchKernelGGL((k_plan<kMaxClusters / 1024, 1024>), dim3(1), dim3(1024), 0, s, d, t,
                       kind, api_nj, allow_small ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_force(const Dev &d, int mode, int src, int K,
                        const RawSrc *raw, const int32_t *list, int role,
                        const NearSpec &nr, int grid, hipStream_t s) {
  ForceArgs A;
  A.d = d;
  A.active = list;
  A.rx = A.rv = A.rm = nullptr;
  A.pred_on = d.pred_on;
  A.role = role;
  A.near = nr.src;
  A.near_c = nr.c;
  if (src == kSrcRaw) {
    if (!raw) return hipErrorInvalidValue;
    A.rx = raw->x;
    A.rv = raw->v;
    A.rm = raw->m;
  }
#define NB_CASE(M, S_, KK)                                    \
  if (mode == M && src == S_ && K == KK)                      \
    return launch_force_t<M, S_, KK>(A, grid, s);
  NB_CASE(kModeFP64, kSrcState, 1)
  NB_CASE(kModeFP64, kSrcState, 2)
  NB_CASE(kModeFP64, kSrcRaw, 1)
  NB_CASE(kModeFP64, kSrcRaw, 2)
  NB_CASE(kModeMixed, kSrcState, 1)
  NB_CASE(kModeMixed, kSrcState, 2)
  NB_CASE(kModeMixed, kSrcRaw, 1)
  NB_CASE(kModeMixed, kSrcRaw, 2)
  NB_CASE(kModeFP64Acc, kSrcState, 1)
  NB_CASE(kModeFP64Acc, kSrcState, 2)
  NB_CASE(kModeFP64Acc, kSrcRaw, 1)
  NB_CASE(kModeFP64Acc, kSrcRaw, 2)
  NB_CASE(kModeMixedAcc, kSrcState, 1)
  NB_CASE(kModeMixedAcc, kSrcState, 2)
  NB_CASE(kModeMixedAcc, kSrcRaw, 1)
  NB_CASE(kModeMixedAcc, kSrcRaw, 2)
  NB_CASE(kModeFP64, kSrcRec, 1)
  NB_CASE(kModeFP64, kSrcRec, 2)
  NB_CASE(kModeMixed, kSrcRec, 1)
  NB_CASE(kModeMixed, kSrcRec, 2)
  NB_CASE(kModeFP64Acc, kSrcRec, 1)
  NB_CASE(kModeFP64Acc, kSrcRec, 2)
  NB_CASE(kModeMixedAcc, kSrcRec, 1)
  NB_CASE(kModeMixedAcc, kSrcRec, 2)
  NB_CASE(kModeMixed64, kSrcState, 1)
  NB_CASE(kModeMixed64, kSrcState, 2)
  NB_CASE(kModeMixed64, kSrcRaw, 1)
  NB_CASE(kModeMixed64, kSrcRaw, 2)
  NB_CASE(kModeMixed64, kSrcRec, 1)
  NB_CASE(kModeMixed64, kSrcRec, 2)
  NB_CASE(kModeMixed64Acc, kSrcState, 1)
  NB_CASE(kModeMixed64Acc, kSrcState, 2)
  NB_CASE(kModeMixed64Acc, kSrcRaw, 1)
  NB_CASE(kModeMixed64Acc, kSrcRaw, 2)
  NB_CASE(kModeMixed64Acc, kSrcRec, 1)
  NB_CASE(kModeMixed64Acc, kSrcRec, 2)
  NB_CASE(kModePot, kSrcState, 1)
#undef NB_CASE
  return hipErrorInvalidValue;
}

int force_grid_size(int mode, int src, int K, int device) {
#define NB_CASE(M, S_, KK) \
  if (mode == M && src == S_ && K == KK) return grid_t<M, S_, KK>(device);
  NB_CASE(kModeFP64, kSrcState, 1)
  NB_CASE(kModeFP64, kSrcState, 2)
  NB_CASE(kModeFP64, kSrcRaw, 1)
  NB_CASE(kModeFP64, kSrcRaw, 2)
  NB_CASE(kModeMixed, kSrcState, 1)
  NB_CASE(kModeMixed, kSrcState, 2)
  NB_CASE(kModeMixed, kSrcRaw, 1)
  NB_CASE(kModeMixed, kSrcRaw, 2)
  NB_CASE(kModeFP64Acc, kSrcState, 1)
  NB_CASE(kModeFP64Acc, kSrcState, 2)
  NB_CASE(kModeFP64Acc, kSrcRaw, 1)
  NB_CASE(kModeFP64Acc, kSrcRaw, 2)
  NB_CASE(kModeMixedAcc, kSrcState, 1)
  NB_CASE(kModeMixedAcc, kSrcState, 2)
  NB_CASE(kModeMixedAcc, kSrcRaw, 1)
  NB_CASE(kModeMixedAcc, kSrcRaw, 2)
  NB_CASE(kModeFP64, kSrcRec, 1)
  NB_CASE(kModeFP64, kSrcRec, 2)
  NB_CASE(kModeMixed, kSrcRec, 1)
  NB_CASE(kModeMixed, kSrcRec, 2)
  NB_CASE(kModeFP64Acc, kSrcRec, 1)
  NB_CASE(kModeFP64Acc, kSrcRec, 2)
  NB_CASE(kModeMixedAcc, kSrcRec, 1)
  NB_CASE(kModeMixedAcc, kSrcRec, 2)
  NB_CASE(kModeMixed64, kSrcState, 1)
  NB_CASE(kModeMixed64, kSrcState, 2)
  NB_CASE(kModeMixed64, kSrcRaw, 1)
  NB_CASE(kModeMixed64, kSrcRaw, 2)
  NB_CASE(kModeMixed64, kSrcRec, 1)
  NB_CASE(kModeMixed64, kSrcRec, 2)
  NB_CASE(kModeMixed64Acc, kSrcState, 1)
  NB_CASE(kModeMixed64Acc, kSrcState, 2)
  NB_CASE(kModeMixed64Acc, kSrcRaw, 1)
  NB_CASE(kModeMixed64Acc, kSrcRaw, 2)
  NB_CASE(kModeMixed64Acc, kSrcRec, 1)
  NB_CASE(kModeMixed64Acc, kSrcRec, 2)
  NB_CASE(kModePot, kSrcState, 1)
#undef NB_CASE
  return 0;
}

hipError_t launch_sym_kick_drift(const Dev &d, double ck, double cd, bool check,
                                 const Tuning &t, hipStream_t s) {
  const int pk = d.C == 1 ? (int)kPlanState : -1;
  if (d.fld.on)
    hipLaunchKernelGGL(k_sym_kick_drift<true>, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, ck,
                       cd, check ? 1 : 0, t, pk);
  else
    hipLaunchKernelGGL(k_sym_kick_drift<false>, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, ck,
                       cd, check ? 1 : 0, t, pk);
  return hipGetLastError();
}

hipError_t launch_sym_kick(const Dev &d, double ck, hipStream_t s) {
  if (d.fld.on)
    hipLaunchKernelGGL(k_sym_kick<true>, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, ck);
  else
    hipLaunchKernelGGL(k_sym_kick<false>, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, ck);
  return hipGetLastError();
}

hipError_t launch_sym_advance(const Dev &d, int64_t dticks, hipStream_t s) {
  const int64_t need = d.n > d.C ? d.n : d.C;
  // the cluster update needs one thread per cluster: C <= 4096 * kWG
  hipLaunchKernelGGL(k_sym_advance, dim3(grid_for(need)), dim3(kWG), 0, s, d, dticks);
  return hipGetLastError();
}

hipError_t launch_records(const Dev &d, int mode, int kind, const RawSrc *raw,
                          bool allow_sb, bool always, bool sb_only, hipStream_t s) {
  RawSrc r{};
  if (raw) r = *raw;
  const int64_t nj = (kind == kPlanApi && r.n_j > 0) ? r.n_j : d.n;
  const dim3 g(grid_for(nj, kWG, 1024)), b(kWG);
  const int sb = allow_sb ? 1 : 0, al = always ? 1 : 0, so = sb_only ? 1 : 0;
  if (mode == kModeMixed || mode == kModeMixedAcc)     // double-single records
    hipLaunchKernelGGL(k_records<kModeMixed>, g, b, 0, s, d, kind, r, sb, al, so);
  else if (mode == kModeMixed64 || mode == kModeMixed64Acc)   // FP64 records, m / m_ref
    hipLaunchKernelGGL(k_records<kModeMixed64>, g, b, 0, s, d, kind, r, sb, al, so);
  else
    hipLaunchKernelGGL(k_records<kModeFP64>, g, b, 0, s, d, kind, r, sb, al, so);
  return hipGetLastError();
}

hipError_t launch_force_sb(const Dev &d, int mode, int K, const RawSrc *raw,
                           const int32_t *list, const NearSpec &nr, int grid, hipStream_t s) {
  ForceArgs A;
  A.d = d;
  A.active = list;
  A.rx = raw ? raw->x : nullptr;
  A.rv = raw ? raw->v : nullptr;
  A.rm = raw ? raw->m : nullptr;
  A.pred_on = d.pred_on;
  A.role = kRoleMain;
  A.near = nr.src;
  A.near_c = nr.c;
  const dim3 g(grid), b(kWG);
#define NB_CASE(M, KK) \
  if (mode == M && K == KK) { hipLaunchKernelGGL((k_force_sb<M, KK>), g, b, prefix_lds_bytes(d.C), s, A); return hipGetLastError(); }
  NB_CASE(kModeFP64, 1)
  NB_CASE(kModeFP64, 2)
  NB_CASE(kModeMixed, 1)
  NB_CASE(kModeMixed, 2)
  NB_CASE(kModeFP64Acc, 1)
  NB_CASE(kModeFP64Acc, 2)
  NB_CASE(kModeMixedAcc, 1)
  NB_CASE(kModeMixedAcc, 2)
  NB_CASE(kModeMixed64, 1)
  NB_CASE(kModeMixed64, 2)
  NB_CASE(kModeMixed64Acc, 1)
  NB_CASE(kModeMixed64Acc, 2)
#undef NB_CASE
  return hipErrorInvalidValue;
}

int force_sb_grid_size(int mode, int K, int device) {
  const void *f = nullptr;
#define NB_CASE(M, KK) \
  if (mode == M && K == KK) f = (const void *)k_force_sb<M, KK>;
  NB_CASE(kModeFP64, 1)
  NB_CASE(kModeFP64, 2)
  NB_CASE(kModeMixed, 1)
  NB_CASE(kModeMixed, 2)
  NB_CASE(kModeFP64Acc, 1)
  NB_CASE(kModeFP64Acc, 2)
  NB_CASE(kModeMixedAcc, 1)
  NB_CASE(kModeMixedAcc, 2)
  NB_CASE(kModeMixed64, 1)
  NB_CASE(kModeMixed64, 2)
  NB_CASE(kModeMixed64Acc, 1)
  NB_CASE(kModeMixed64Acc, 2)
#undef NB_CASE
  if (!f) return 0;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kWG, 0) != hipSuccess) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    cus = 256;
  if (per_cu < 1) per_cu = 1;
  return per_cu * cus;
}

hipError_t launch_sum_and_flag(const Dev &d, const int32_t *list, int64_t na_host,
                               float refine_ratio, const NearSpec &nr, bool theta_out,
                               const Tuning &t1, int ref_kind, int64_t api_nj, bool append,
                               hipStream_t s) {
  const int64_t cap = na_host >= 0 ? na_host : d.cap_active;
  // at most one wave per entry, grid-stride
  const dim3 g(grid_for(cap * 64, kWG, 4096)), b(kWG);
  const size_t lds = prefix_lds_bytes(d.C);
  const int th = theta_out ? 1 : 0;
  // one cluster with a fused plan (block steps): the flagged entries are
  // appended and planned by the sum launch itself
  const bool app = append && plan_fused(d) && refine_ratio > 0.0f && !theta_out;
  if (app)
    hipLaunchKernelGGL(k_sum_flag<true>, g, b, lds, s, d, list, refine_ratio, nr.c, nr.src, th,
                       t1, ref_kind);
  else
    hipLaunchKernelGGL(k_sum_flag<false>, g, b, lds, s, d, list, refine_ratio, nr.c, nr.src, th,
                       t1, ref_kind);
  if (refine_ratio > 0.0f && !theta_out && !app) {
    if (d.nblk <= kFusedScan) {
      hipLaunchKernelGGL(k_rscatter<true>, dim3(d.nblk), dim3(kWG), 0, s, d, list, na_host, t1,
                         plan_fused(d) ? ref_kind : -1, api_nj);
    } else {
      hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d, (const int32_t *)d.flag_cnt);
      hipLaunchKernelGGL(k_rscatter<false>, dim3(d.nblk), dim3(kWG), 0, s, d, list, na_host,
                         t1, -1, api_nj);
    }
  }
  return hipGetLastError();
}

hipError_t launch_refine_finalize(const Dev &d, const CorrectSpec *corr, hipStream_t s) {
  const int rb = grid_for(d.cap_active * 64, kWG, 512);
  const dim3 b(kWG);
  const CorrectSpec cs = corr ? *corr : CorrectSpec{};
  // the corrector's blocks: one thread per active entry
  const int cb = corr ? grid_for(d.cap_active, kWG, 2048) : 0;
  if (!corr)
    hipLaunchKernelGGL((k_ref_final<false, false>), dim3(rb), b, 0, s, d, rb, cs);
  else if (d.fld.on)
    hipLaunchKernelGGL((k_ref_final<true, true>), dim3(rb + cb), b, 0, s, d, rb, cs);
  else
    hipLaunchKernelGGL((k_ref_final<true, false>), dim3(rb + cb), b, 0, s, d, rb, cs);
  return hipGetLastError();
}

hipError_t launch_vref(const Dev &d, const RawSrc *raw, hipStream_t s) {
  RawSrc r{};
  if (raw) r = *raw;
  if (raw && !raw->v) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vref, dim3(d.C), dim3(kWG), 0, s, d, r);
  return hipGetLastError();
}

hipError_t launch_correct(const Dev &d, double eta, double dt_shared,
                          int level_min, int level_max, hipStream_t s) {
  const dim3 g(grid_for((int64_t)d.cap_active * 64, kWG, 4096)), b(kWG);
  const size_t lds = prefix_lds_bytes(d.C);
  if (d.fld.on)
    hipLaunchKernelGGL(k_sum_correct<true>, g, b, lds, s, d, eta, dt_shared, level_min,
                       level_max);
  else
    hipLaunchKernelGGL(k_sum_correct<false>, g, b, lds, s, d, eta, dt_shared, level_min,
                       level_max);
  return hipGetLastError();
}

hipError_t launch_init_levels(const Dev &d, double eta_start, double dt_shared,
                              int level_min, int level_max, hipStream_t s) {
  const dim3 g((unsigned)((d.n + kWG - 1) / kWG));
  if (d.fld.on)
    hipLaunchKernelGGL(k_init_levels<true>, g, dim3(kWG), 0, s, d, eta_start, dt_shared,
                       level_min, level_max);
  else
    hipLaunchKernelGGL(k_init_levels<false>, g, dim3(kWG), 0, s, d, eta_start, dt_shared,
                       level_min, level_max);
  return hipGetLastError();
}

hipError_t launch_api_group(const Dev &d, const RawSrc &r, const Tuning &t, hipStream_t s) {
  int64_t need = r.n_active > d.C + 1 ? r.n_active : d.C + 1;
  hipLaunchKernelGGL(k_api_group, dim3((unsigned)((need + kWG - 1) / kWG)),
                     dim3(kWG), 0, s, d, r.i_active, r.n_active, t, r.n_j);
  return hipGetLastError();
}

hipError_t launch_api_finalize(const Dev &d, const RawSrc &r, hipStream_t s) {
  hipLaunchKernelGGL(k_api_finalize, dim3(grid_for(r.n_active)), dim3(kWG), 0,
                     s, d, r.n_active, r.acc, r.jerk);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const Dev &d, hipStream_t s) {
  if (d.fld.on)
    hipLaunchKernelGGL(k_energy_reduce<true>, dim3(d.C), dim3(kWG), 0, s, d);
  else
    hipLaunchKernelGGL(k_energy_reduce<false>, dim3(d.C), dim3(kWG), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_set_word64(int64_t *p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_word64, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill32, dim3(grid_for(n)), dim3(kWG), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_get_state(const Dev &d, double *x, double *v, double *a,
                            double *jk, int64_t *tick, int8_t *level,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_get_state, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, x, v,
                     a, jk, tick, level);
  return hipGetLastError();
}

hipError_t launch_set_state(const Dev &d, const double *x, const double *v,
                            const double *a, const double *jk,
                            const int64_t *tick, const int8_t *level,
                            int level_min, int level_max, hipStream_t s) {
  // T and hist are cleared by the caller (fill kernels) beforehand
  hipLaunchKernelGGL(k_set_state1, dim3(grid_for(d.n)), dim3(kWG), 0, s, d, x,
                     v, a, jk, tick, level, level_min, level_max);
  int64_t need = d.n > d.C ? d.n : d.C;
  hipLaunchKernelGGL(k_set_state2, dim3(grid_for(need)), dim3(kWG), 0, s, d);
  return hipGetLastError();
}

}  // namespace nbk
