// Shared device helpers of the tdgemm HIP library (gfx950).
//
// Compile with -ffp-contract=off: every floating-point expression below is
// evaluated operation by operation in the order written, with fused
// multiply-adds only where __builtin_fma is spelled out.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tdgemm.h"

namespace tdg {

constexpr int kThreads = 256;          // threads per workgroup of every kernel
constexpr int kWave = 64;              // CDNA wavefront width
constexpr double kDUnavailable = 1e300;  // D of an option the calibration cannot supply
constexpr int kMaxR = 512;             // calibration grid points
// Fourth word of a raw buffer resource on gfx9: 32-bit data format, no swizzle.
constexpr int kBufWord3 = 0x00020000;

// Workgroup barrier that orders LDS accesses only: global loads a thread has in
// flight stay in flight (a plain __syncthreads also waits for them, which
// would cut a software prefetch short at every barrier). Use it where threads
// share data through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Compensated sums. A running sum is a pair (s, c): s the rounded sum, c the
// accumulated rounding errors (each obtained exactly by TwoSum). s + c rounded
// once is the exactly rounded sum except when the exact value lies within about
// n^2 2^-106 |sum| of a rounding boundary; certified_round() below detects that
// case and the callers then sum exactly.
struct CSum {
  double s, c;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ CSum csum_add(CSum x, double v) {
  double s, e;
  two_sum(x.s, v, s, e);
  return CSum{s, x.c + e};
}

__device__ __forceinline__ CSum csum_merge(CSum x, CSum y) {
  double s, e;
  two_sum(x.s, y.s, s, e);
  return CSum{s, (x.c + y.c) + e};
}

__device__ __forceinline__ double csum_value(CSum x) { return x.s + x.c; }

// Butterfly merge over the 64 lanes, then lane 0's pair broadcast so every lane
// holds the same (s, c).
__device__ __forceinline__ CSum wave_csum_pair(CSum x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    CSum y{__shfl_xor(x.s, off), __shfl_xor(x.c, off)};
    x = csum_merge(x, y);
  }
  return CSum{__shfl(x.s, 0), __shfl(x.c, 0)};
}

// ---------------------------------------------------------------------------
// Exactly rounded sums by construction. A compensated pair (s, c) of n terms
// whose exact sum S is at least as large as the sum of their magnitudes up to
// a factor 1 + 2^-50 (non-negative terms, or squares split exactly into a
// rounded square and its error) satisfies |S - (s + c)| <= ~(n 2^-53)^2 |S|.
// exact_bound() is n^2 2^-100 |s + c|, a generous multiple of that.
// certified_round() returns r = fl(s + c) and whether r is certainly the
// exactly rounded S: S then lies strictly inside r's rounding interval. Where
// it does not, the caller sums the terms again exactly in a long accumulator
// (below) and rounds once to nearest, ties to even.
__device__ __forceinline__ double exact_bound(int64_t n, double r) {
  return (((double)n * (double)n) * 0x1p-100) * fabs(r);
}

__device__ __forceinline__ bool certified_round(double s, double c, int64_t n, double &r) {
  double t;
  two_sum(s, c, r, t);                            // r + t = s + c exactly
  if (r == 0.0 || !isfinite(r)) return true;      // all terms zero, or overflow either way
  const double ar = fabs(r);
  const int64_t bits = __double_as_longlong(ar);
  // distance from r to its neighbour on the side of t
  const bool away = (t >= 0.0) == (r > 0.0);
  const double gap = away ? __longlong_as_double(bits + 1) - ar : ar - __longlong_as_double(bits - 1);
  return fabs(t) + exact_bound(n, r) < 0.5 * gap;
}

// Exact long accumulator: the terms' exact sum as signed 64-bit limbs, limb k
// holding digits of weight 2^(32 k - 1074), so that every finite double is a
// whole number of units 2^-1074. A term adds its 53-bit significand, split into
// three 32-bit pieces, to three limbs with LDS atomics (any order, any number of
// threads); each limb stays far from overflow for fewer than 2^28 terms.
// lacc_round() then propagates the carries and rounds once to nearest, ties to
// even. 68 limbs cover 2176 bits: the 2098 of binary64 plus the carries.
constexpr int kAccLimbs = 68;

__device__ __forceinline__ void lacc_add(int64_t *acc, double x) {
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const int ex = (int)((bits >> 52) & 0x7ff);
  uint64_t m = bits & ((uint64_t(1) << 52) - 1);
  if (ex != 0) m |= uint64_t(1) << 52;
  if (m == 0) return;
  const int b = ex == 0 ? 0 : ex - 1;              // weight of m's unit bit, in units 2^-1074
  const int k = b >> 5, sh = b & 31;
  const uint64_t lo = m << sh;                      // bits 0..63 of m 2^sh
  const uint64_t hi = sh ? (m >> (64 - sh)) : 0;    // bits 64..84
  const int64_t d0 = (int64_t)(lo & 0xffffffffu), d1 = (int64_t)(lo >> 32), d2 = (int64_t)hi;
  const bool neg = (bits >> 63) != 0;
  atomicAdd((unsigned long long *)&acc[k], (unsigned long long)(neg ? -d0 : d0));
  atomicAdd((unsigned long long *)&acc[k + 1], (unsigned long long)(neg ? -d1 : d1));
  atomicAdd((unsigned long long *)&acc[k + 2], (unsigned long long)(neg ? -d2 : d2));
}

// One thread: the accumulated sum rounded once to nearest, ties to even. The
// limbs are normalised in place (digits in [0, 2^32), the magnitude if the sum
// is negative). Out of line and with rolled loops: it is the rare path of every
// exact sum, and inlined copies of the unrolled limb loops made the plan kernel
// three times longer.
__device__ __noinline__ double lacc_round(int64_t *acc) {
  int64_t carry = 0;
#pragma unroll 1
  for (int k = 0; k < kAccLimbs; ++k) {
    const int64_t v = acc[k] + carry;
    carry = v >> 32;                                // floor division by 2^32
    acc[k] = v - (carry << 32);
  }
  const bool neg = carry < 0;                       // the sum is carry 2^(32 kAccLimbs) + digits
  if (neg) {                                        // magnitude: two's complement of the digits
    int64_t c = 1;
#pragma unroll 1
    for (int k = 0; k < kAccLimbs; ++k) {
      const int64_t v = (0xffffffffll - acc[k]) + c;
      c = v >> 32;
      acc[k] = v & 0xffffffffll;
    }
  }
  int h = kAccLimbs - 1;
  while (h >= 0 && acc[h] == 0) --h;
  if (h < 0) return 0.0;
  const int lead = 32 * h + 31 - __builtin_clz((unsigned)acc[h]);   // top bit, in units 2^-1074
  double r;
  if (lead < 53) {                                  // at most 53 bits: exact (subnormal or small normal)
    const uint64_t n = (uint64_t)acc[0] | ((uint64_t)acc[1] << 32);
    r = ldexp((double)n, -1074);
  } else {
    const int lo = lead - 63;                       // window of bits lo .. lead
    uint64_t w = 0;
    for (int q = 0; q < 3; ++q) {
      const int k = (lo >> 5) + q;
      const uint64_t d = (k >= 0 && k < kAccLimbs) ? (uint64_t)acc[k] : 0;
      const int pos = 32 * q - (lo & 31);           // where digit k's bit 0 lands in the window
      if (pos >= 0) { if (pos < 64) w |= d << pos; }
      else w |= d >> (-pos);
    }
    uint64_t mant = w >> 11;                        // 53 bits, top one set
    const bool half = (w >> 10) & 1;
    bool sticky = (w & 0x3ff) != 0;
    if (lo > 0) {                                   // bits below the window
      const int kl = lo >> 5;
      if ((uint64_t)acc[kl] & ((uint64_t(1) << (lo & 31)) - 1)) sticky = true;
      for (int k = 0; k < kl && !sticky; ++k) sticky = acc[k] != 0;
    }
    if (half && (sticky || (mant & 1))) mant += 1;  // 2^53 stays exact
    r = ldexp((double)mant, lo + 11 - 1074);
  }
  return neg ? -r : r;
}

// Orders this wavefront's LDS accesses around the point of the call.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A compensated pair that also records whether every addition into c was
// exact. If so, s + c is the exact sum (each TwoSum error is exact), and
// rounding it once gives the exactly rounded sum with no certificate: this is
// the common case of a few terms whose exact sum needs only a few bits beyond
// s, and it includes exact ties, which the certificate can never decide.
struct XSum {
  double s, c;
  int exact;
};

__device__ __forceinline__ XSum xsum_add(XSum x, double v) {
  double s, e, c, ec;
  two_sum(x.s, v, s, e);
  two_sum(x.c, e, c, ec);
  return XSum{s, c, x.exact & (ec == 0.0 ? 1 : 0)};
}

__device__ __forceinline__ XSum xsum_merge(XSum x, XSum y) {
  double s, e, c1, e1, c, e2;
  two_sum(x.s, y.s, s, e);
  two_sum(x.c, y.c, c1, e1);
  two_sum(c1, e, c, e2);
  return XSum{s, c, x.exact & y.exact & ((e1 == 0.0 && e2 == 0.0) ? 1 : 0)};
}

// Partner values for step OFF of a wavefront all-reduce whose steps run in the
// order 1, 2, 4, 8, 16, 32. Steps 1 and 2 swap neighbours within a quad and
// steps 4 and 8 mirror each half-row and row, all as DPP moves; by then every
// lane of a group already holds its group's result, so any lane of the partner
// group will do. Steps 16 and 32 use ds_bpermute. Every lane must be active.
template <int OFF>
__device__ __forceinline__ int lane_partner(int v) {
  if constexpr (OFF == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);    // quad_perm 1,0,3,2
  else if constexpr (OFF == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
  else if constexpr (OFF == 4) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false); // row_half_mirror
  else if constexpr (OFF == 8) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false); // row_mirror
  else return __shfl_xor(v, OFF);
}
template <int OFF>
__device__ __forceinline__ double lane_partner(double v) {
  const int64_t b = __double_as_longlong(v);
  const int lo = lane_partner<OFF>((int)(uint32_t)b), hi = lane_partner<OFF>((int)(b >> 32));
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
template <int OFF>
__device__ __forceinline__ XSum xsum_step(XSum x) {
  return xsum_merge(x, XSum{lane_partner<OFF>(x.s), lane_partner<OFF>(x.c), lane_partner<OFF>(x.exact)});
}
__device__ __forceinline__ double lane0(double v) {
  const int64_t b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 0);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(b >> 32), 0);
  return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// Exactly rounded sum of v[0..TT) over the 64 lanes of a wavefront; every lane
// gets the same value. The merges may run in any order: the result is the
// exactly rounded sum either way. scr: this wavefront's LDS scratch of at least
// kAccLimbs doubles, used only when the compensated sum is neither exact nor
// certified. Every lane must be active.
template <int TT>
__device__ __forceinline__ double wave_sum_exact(const double (&v)[TT], double *scr) {
  const int lane = threadIdx.x & (kWave - 1);
  XSum x{0.0, 0.0, 1};
#pragma unroll
  for (int t = 0; t < TT; ++t) x = xsum_add(x, v[t]);
  x = xsum_step<1>(x);
  x = xsum_step<2>(x);
  x = xsum_step<4>(x);
  x = xsum_step<8>(x);
  x = xsum_step<16>(x);
  x = xsum_step<32>(x);
  x = XSum{lane0(x.s), lane0(x.c), __builtin_amdgcn_readlane(x.exact, 0)};
  double r;
  if (x.exact && isfinite(x.s)) return x.s + x.c;
  if (certified_round(x.s, x.c, (int64_t)kWave * TT, r)) return r;
  int64_t *acc = reinterpret_cast<int64_t *>(scr);
  wave_sync_lds();
  for (int k = lane; k < kAccLimbs; k += kWave) acc[k] = 0;
  wave_sync_lds();
#pragma unroll
  for (int t = 0; t < TT; ++t) lacc_add(acc, v[t]);
  wave_sync_lds();
  if (lane == 0) r = lacc_round(acc);
  r = __shfl(r, 0);
  wave_sync_lds();
  return r;
}

// ---------------------------------------------------------------------------
// Plan arithmetic: the paper's formulas in the operation order written.

// p = ceil(log2(2 R_safe + u_safe)): z = 2^-p is the largest power of two
// satisfying eq. (15). Exact: v is an integer below 2^53 and frexp is exact.
__device__ __forceinline__ int packing_exponent(double r_safe, double u_safe) {
  double v = 2.0 * r_safe + u_safe;
  int e;
  double m = frexp(v, &e);
  return (m == 0.5) ? e - 1 : e;
}

struct BlockMoments {
  double amax;    // max{|min|, max}
  double sigma;   // sqrt(sumsq / n)
};

__device__ __forceinline__ BlockMoments moments(const tdgemm_block_stats &st) {
  BlockMoments b;
  b.amax = fmax(fabs(st.mn), st.mx);
  b.sigma = sqrt(st.sumsq / (double)st.n);
  return b;
}

// Normalised noise at the eq. (26) companders (eq. 27 read from eqs. 19 and 21):
// c_tot/(6 s_a s_b) + c_tot^2/(144 s_a^2 s_b^2) + s^2 c_tot^2/(L s_a^2 s_b^2).
__device__ __forceinline__ double nsr_exact(double L_eff, double amax_a, double amax_b, double ss,
                                            double r, double s) {
  double ctot = ((L_eff * amax_a) * amax_b) / r;
  double t1 = ctot / (6.0 * ss);
  double t2 = (ctot * ctot) / (144.0 * (ss * ss));
  double t3 = ((s * s) * (ctot * ctot)) / (L_eff * (ss * ss));
  return (t1 + t2) + t3;
}

// Settings of one pair (the fields of tdgemm_pair).
__device__ __forceinline__ tdgemm_pair option_native() {
  tdgemm_pair o;
  o.c_a = 1.0; o.c_b = 1.0; o.inv = 1.0; o.d = 0.0; o.r_max = 0.0; o.s_rep = 0.0;
  o.q_a = 0.0; o.q_b = 0.0; o.w = 1; o.p = 0;
  return o;
}

__device__ __forceinline__ tdgemm_pair option_zero(int W, double u_safe) {
  tdgemm_pair o;
  o.c_a = 0.0; o.c_b = 0.0; o.inv = 0.0; o.d = 0.0; o.r_max = 0.0; o.s_rep = 0.0;
  o.q_a = 0.0; o.q_b = 0.0; o.w = W; o.p = packing_exponent(0.0, u_safe);
  return o;
}

// Eq. (21) at companders c_a, c_b: L[(s_a s_nb)^2 + (s_b s_na)^2 + (s_na s_nb)^2]
// + (s / (c_a c_b))^2 with s_n = 1 / (c sqrt 12).
__device__ __forceinline__ double noise_eq21(double L_eff, double s_a, double s_b, double c_a,
                                             double c_b, double s_rep) {
  const double sqrt12 = 3.4641016151377544;   // correctly rounded sqrt(12)
  double rep = s_rep / (c_a * c_b);
  double na = 1.0 / (c_a * sqrt12);
  double nb = 1.0 / (c_b * sqrt12);
  double q = L_eff * (((s_a * nb) * (s_a * nb) + (s_b * na) * (s_b * na)) + (na * nb) * (na * nb));
  return q + rep * rep;
}

// Eqs. (24), (26), (15), (21) at packing W and range r_max.
__device__ __forceinline__ tdgemm_pair option_at(int W, double L_eff, const BlockMoments &a,
                                                 const BlockMoments &b, double r_max, double s_rep,
                                                 double u_safe) {
  tdgemm_pair o;
  double ctot = ((L_eff * a.amax) * b.amax) / r_max;
  o.c_a = sqrt(b.sigma / (a.sigma * ctot));
  o.c_b = sqrt(a.sigma / (b.sigma * ctot));
  o.q_a = rint(o.c_a * a.amax);
  o.q_b = rint(o.c_b * b.amax);
  double r_safe = (L_eff * o.q_a) * o.q_b;
  o.p = packing_exponent(r_safe, u_safe);
  o.d = noise_eq21(L_eff, a.sigma, b.sigma, o.c_a, o.c_b, s_rep);
  o.inv = 1.0 / (o.c_a * o.c_b);
  o.r_max = r_max;
  o.s_rep = s_rep;
  o.w = W;
  return o;
}

// Prop. 3 at packing W and range r_max: the eq. (22) companders (+ root) reaching
// the expected subblock SNR S, given as pw = 10^(S/10) (computed on the host);
// D_QvR of eq. (23) in the form 12 s_a^2 s_b^2 / 10^(S/10) - c_tot^2 (1 + (12 s)^2 / L) / 12.
// Where eq. (25) fails the double root is taken: the eq. (26) companders.
__device__ __forceinline__ tdgemm_pair option_target(int W, double L_eff, const BlockMoments &a,
                                                     const BlockMoments &b, double r_max,
                                                     double s_rep, double pw, double u_safe) {
  const double sqrt2 = 1.4142135623730951;    // correctly rounded sqrt(2)
  double ctot = ((L_eff * a.amax) * b.amax) / r_max;
  double ss = a.sigma * b.sigma;
  double rs = 12.0 * s_rep;
  double d = ((12.0 * ss) * ss) / pw - ((ctot * ctot) * (1.0 + (rs * rs) / L_eff)) / 12.0;
  double disc = d * d - (((((4.0 * a.sigma) * a.sigma) * b.sigma) * b.sigma) * ctot) * ctot;
  tdgemm_pair o;
  if (d < ((2.0 * a.sigma) * b.sigma) * ctot || disc < 0.0) {       // eq. (25) fails
    o.c_a = sqrt(b.sigma / (a.sigma * ctot));
    o.c_b = sqrt(a.sigma / (b.sigma * ctot));
  } else {
    double root = sqrt(d + sqrt(disc));
    o.c_a = root / ((sqrt2 * a.sigma) * ctot);
    o.c_b = (sqrt2 * a.sigma) / root;
  }
  o.q_a = rint(o.c_a * a.amax);
  o.q_b = rint(o.c_b * b.amax);
  double r_safe = (L_eff * o.q_a) * o.q_b;
  o.p = packing_exponent(r_safe, u_safe);
  o.d = noise_eq21(L_eff, a.sigma, b.sigma, o.c_a, o.c_b, s_rep);
  o.inv = 1.0 / (o.c_a * o.c_b);
  o.r_max = r_max;
  o.s_rep = s_rep;
  o.w = W;
  return o;
}

// Per-block companders c = Q / max|X| (same integers for every pair of a block).
__device__ __forceinline__ tdgemm_pair option_separable(int W, double L_eff, const BlockMoments &a,
                                                        const BlockMoments &b, double q,
                                                        double u_safe) {
  tdgemm_pair o;
  o.c_a = q / a.amax;
  o.c_b = q / b.amax;
  o.q_a = rint(o.c_a * a.amax);
  o.q_b = rint(o.c_b * b.amax);
  double r_safe = (L_eff * o.q_a) * o.q_b;
  o.p = packing_exponent(r_safe, u_safe);
  o.d = noise_eq21(L_eff, a.sigma, b.sigma, o.c_a, o.c_b, 0.0);
  o.inv = 1.0 / (o.c_a * o.c_b);
  o.r_max = r_safe;
  o.s_rep = 0.0;
  o.w = W;
  return o;
}

// Index (into the full table) of the first minimum of nsr_exact over the
// table points with finite s, or -1 if there is none.
//
// Only non-dominated points are scanned: a point k is dominated when a point
// k' with a larger R has s[k'] / R[k'] <= s[k] / R[k]; then every term of the
// noise is smaller at k' (the first two strictly, by the grid spacing), so k
// can never be the first minimum. `idx` lists the remaining points in
// ascending R; `fr` and `fs2` hold 1/R and s^2 in FP32. An FP32 pass finds the
// approximate minimum (relative error below 1e-6); the exact formula is then
// evaluated, in ascending order, at every point within a relative 1e-5 of it,
// so the result equals a full exact scan.
//
// The scan may be shared by LP lanes (a power of two; the aligned group of LP
// lanes holding the same pair): lane `sub` of the group scans the points
// sub, sub + LP, ...; the FP32 minimum and then the exact (value, index) pair,
// lowest index on equal values, are reduced over the group. Minima are exact,
// so every group lane gets the serial scan's result.
__device__ __forceinline__ int argmin_nsr(double L_eff, const BlockMoments &a, const BlockMoments &b,
                                          const double *r, const double *s, const short *idx,
                                          const float *fr, const float *fs2, int cnt,
                                          int sub = 0, int LP = 1) {
  const double ss = a.sigma * b.sigma;
  const float x0 = (float)(((L_eff * a.amax) * b.amax) / ss);   // c_tot * R / (s_a s_b)
  const float invL = 1.0f / (float)L_eff;
  float best = INFINITY;
#pragma unroll 4
  for (int i = sub; i < cnt; i += LP) {
    const float x = x0 * fr[i];
    best = fminf(best, x * ((1.0f / 6.0f) + x * ((1.0f / 144.0f) + fs2[i] * invL)));
  }
  for (int off = 1; off < LP; off <<= 1) best = fminf(best, __shfl_xor(best, off));
  const float thr = (best < INFINITY) ? best * (1.0f + 1e-5f) : INFINITY;
  int kbest = -1;
  double vbest = INFINITY;
#pragma unroll 4
  for (int i = sub; i < cnt; i += LP) {
    const float x = x0 * fr[i];
    const float v = x * ((1.0f / 6.0f) + x * ((1.0f / 144.0f) + fs2[i] * invL));
    if (v <= thr) {
      const int k = idx[i];
      const double e = nsr_exact(L_eff, a.amax, b.amax, ss, r[k], s[k]);
      if (e < vbest) { vbest = e; kbest = k; }
    }
  }
  for (int off = 1; off < LP; off <<= 1) {
    const double ov = __shfl_xor(vbest, off);
    const int ok = __shfl_xor(kbest, off);
    if (ov < vbest || (ov == vbest && ok >= 0 && (kbest < 0 || ok < kbest))) { vbest = ov; kbest = ok; }
  }
  return kbest;
}

// ---------------------------------------------------------------------------
// Non-dominated calibration points per W row (W = 2, 3, 4), ascending R: grid
// index, 1/R and s^2 in FP32 (see argmin_nsr). Built by the statistics launch.
struct PlanTable {
  int32_t cnt[4];
  int16_t idx[3][kMaxR];
  float fr[3][kMaxR];
  float fs2[3][kMaxR];
};

// Workspace layout shared by the host code and the kernels.
struct Layout {
  int64_t nI, nL, nJ, n_pairs;
  size_t off_stats_a, off_stats_b, off_pairs, off_budget, off_target, off_table, off_part, total;
  int64_t gsize, ngroups;     // subblocks per group of the l-sum, and the number of groups
};

// Subblocks per group of the l-sum for k_split groups requested (0 or 1: all).
__host__ __device__ inline int64_t group_size(int64_t nl, int64_t k_split) {
  if (k_split <= 1 || nl <= 0) return nl > 0 ? nl : 1;
  const int64_t s = (nl + k_split - 1) / k_split;
  return s > 0 ? s : 1;
}

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// part_elem: bytes per element of the partial results of a split l-sum (0: none).
__host__ inline Layout make_layout(int64_t M, int64_t N, int64_t K, int L, int64_t k_split = 1,
                                   size_t part_elem = 0) {
  Layout ly;
  ly.nI = (M + L - 1) / L;
  ly.nL = (K + L - 1) / L;
  ly.nJ = (N + L - 1) / L;
  ly.n_pairs = ly.nI * ly.nL * ly.nJ;
  size_t off = 0;
  ly.off_stats_a = off; off = align256(off + sizeof(tdgemm_block_stats) * ly.nI * ly.nL);
  ly.off_stats_b = off; off = align256(off + sizeof(tdgemm_block_stats) * ly.nL * ly.nJ);
  ly.off_pairs = off;   off = align256(off + sizeof(tdgemm_pair) * ly.n_pairs);
  ly.off_budget = off;  off = align256(off + sizeof(double) * ly.nI * ly.nJ);
  ly.off_target = off;  off = align256(off + sizeof(double) * ly.nI * ly.nJ);
  ly.off_table = off;   off = align256(off + sizeof(PlanTable));
  ly.gsize = group_size(ly.nL, k_split);
  ly.ngroups = ly.nL > 0 ? (ly.nL + ly.gsize - 1) / ly.gsize : 1;
  ly.off_part = off;
  if (ly.ngroups > 1) off = align256(off + part_elem * (size_t)ly.ngroups * (size_t)M * (size_t)N);
  ly.total = off;
  return ly;
}

// Problem description as the kernels see it (passed by value).
struct Problem {
  int64_t M, N, K, lda, ldb, ldc;
  int64_t nI, nL, nJ;
  int L;
};

}  // namespace tdg
