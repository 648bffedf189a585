// Block statistics (Sec. 3, Sec. 5.B) and the per-pair plan with inner-kernel
// pruning (Sec. 5.B, Sec. 6).
#include "common.h"
#include "kernels.h"

namespace tdg {

// ---------------------------------------------------------------------------
// Block statistics. The result of a block does not depend on the order in
// which its elements are visited (min and max are exact, the sum of squares is
// exactly rounded), so every block is read in its stored layout: a transposed
// operand is the same set of elements.

struct StatAcc {
  double mn, mx;
  CSum s;
};

__device__ __forceinline__ void stat_add(StatAcc &a, double x) {
  a.mn = fmin(a.mn, x);
  a.mx = fmax(a.mx, x);
  const double p = x * x;
  const double pe = __builtin_fma(x, x, -p);     // x^2 = p + pe exactly
  a.s = csum_add(a.s, p);
  a.s.c = a.s.c + pe;
}

__device__ __forceinline__ StatAcc stat_merge(const StatAcc &a, const StatAcc &b) {
  return StatAcc{fmin(a.mn, b.mn), fmax(a.mx, b.mx), csum_merge(a.s, b.s)};
}

__device__ __forceinline__ StatAcc stat_shfl_xor(const StatAcc &a, int off) {
  return StatAcc{__shfl_xor(a.mn, off), __shfl_xor(a.mx, off),
                 CSum{__shfl_xor(a.s.s, off), __shfl_xor(a.s.c, off)}};
}

// One workgroup: the stored block of vr x vc valid elements at X (leading
// dimension ld). A full block whose rows start on 16-byte boundaries is read
// with 16-byte loads, each half of them issued before its first use; other
// blocks element by element with bounds checks. The statistics do not depend
// on the order of the terms (min, max and an exactly rounded sum).
template <typename T, int L>
__device__ __forceinline__ void block_stats(const T *__restrict__ X, int64_t ld, int vr, int vc,
                                            tdgemm_block_stats *out) {
  constexpr int V = 16 / (int)sizeof(T);            // elements per 16-byte load
  constexpr int RV = L / V;                         // loads per row
  constexpr int NV = L * L / V / kThreads;          // loads per thread
  // FP32 inputs: every square is exact in FP64, and the first pass already
  // sums them as exact compensated pairs (below), so ties need no second pass
  constexpr bool kX = std::is_same<T, float>::value;
  typedef T vec_t __attribute__((ext_vector_type(V)));
  const int tid = threadIdx.x;
  StatAcc acc0{INFINITY, -INFINITY, CSum{0.0, 0.0}}, acc1 = acc0;
  XSum x0{0.0, 0.0, 1}, x1 = x0;
  auto add = [&](StatAcc &acc, XSum &x, double v) {
    if constexpr (kX) {
      acc.mn = fmin(acc.mn, v);
      acc.mx = fmax(acc.mx, v);
      x = xsum_add(x, v * v);
    } else {
      stat_add(acc, v);
    }
  };
  const bool vec = vr == L && vc == L && ((uintptr_t)X % 16) == 0 &&
                   ((ld * (int64_t)sizeof(T)) % 16) == 0;
  if (vec) {
    // two halves where the count allows: fewer registers, five workgroups per
    // CU instead of four for FP64 (3.5 us less at 4096^2, 6.0 TB/s)
    constexpr int NP = (NV % 2 == 0) ? 2 : 1;
    constexpr int NH = NV / NP;
#pragma unroll 1
    for (int h = 0; h < NP; ++h) {
      vec_t v[NH];
#pragma unroll
      for (int q = 0; q < NH; ++q) {
        const int e = tid + kThreads * (q + h * NH);
        v[q] = *reinterpret_cast<const vec_t *>(X + (int64_t)(e / RV) * ld + (e % RV) * V);
      }
#pragma unroll
      for (int q = 0; q < NH; ++q)
#pragma unroll
        for (int c = 0; c < V; ++c) {
          if (q & 1) add(acc1, x1, (double)v[q][c]);
          else       add(acc0, x0, (double)v[q][c]);
        }
    }
  } else {
    for (int e = tid; e < L * L; e += kThreads) {
      const int r = e / L, c = e - (e / L) * L;
      if (r < vr && c < vc) add(acc0, x0, (double)X[(int64_t)r * ld + c]);
    }
  }
  StatAcc acc = stat_merge(acc0, acc1);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc = stat_merge(acc, stat_shfl_xor(acc, off));
  __shared__ StatAcc s_w[kThreads / kWave];
  __shared__ double s_sum;
  __shared__ int s_certified;
  __shared__ double s_xs[kThreads / kWave], s_xc[kThreads / kWave];
  __shared__ int s_xe[kThreads / kWave];
  // exact compensated pairs of the lanes, merged over the wavefront and then the
  // workgroup; thread 0 gets the workgroup's pair
  auto merge_x = [&](XSum x) {
    x = xsum_step<1>(x);
    x = xsum_step<2>(x);
    x = xsum_step<4>(x);
    x = xsum_step<8>(x);
    x = xsum_step<16>(x);
    x = xsum_step<32>(x);
    if ((tid & (kWave - 1)) == 0) {
      s_xs[tid / kWave] = x.s;
      s_xc[tid / kWave] = x.c;
      s_xe[tid / kWave] = x.exact;
    }
    __syncthreads();
    XSum t{s_xs[0], s_xc[0], s_xe[0]};
    for (int q = 1; q < kThreads / kWave; ++q) t = xsum_merge(t, XSum{s_xs[q], s_xc[q], s_xe[q]});
    return t;
  };
  if ((tid & (kWave - 1)) == 0) s_w[tid / kWave] = acc;
  XSum tx{0.0, 0.0, 0};
  if constexpr (kX) tx = merge_x(xsum_merge(x0, x1));
  __syncthreads();
  if (tid == 0) {
    StatAcc t = s_w[0];
    for (int q = 1; q < kThreads / kWave; ++q) t = stat_merge(t, s_w[q]);
    double r;
    if constexpr (kX) {
      // one exact term per valid element; the certificate covers inexact pairs
      if (tx.exact && isfinite(tx.s)) {
        s_certified = 1;
        r = tx.s + tx.c;
      } else {
        s_certified = certified_round(tx.s, tx.c, (int64_t)vr * vc, r) ? 1 : 0;
      }
    } else {
      // 2 terms (rounded square and its error) per valid element
      s_certified = certified_round(t.s.s, t.s.c, 2 * (int64_t)vr * vc, r) ? 1 : 0;
    }
    s_sum = r;
    s_w[0] = t;
  }
  __syncthreads();
  if (!kX && !s_certified) {
    // The sum lies too close to a rounding boundary for the compensated pair to
    // decide (an exact tie, say, which data of few significant bits make
    // common). A second pass sums the squares, split exactly into their rounded
    // values and errors, as compensated pairs that record whether every
    // addition into the correction was exact; if so, the pair holds the exact
    // sum and one rounding gives it.
    XSum x{0.0, 0.0, 1};
    for (int e = tid; e < L * L; e += kThreads) {
      const int r = e / L, c = e - (e / L) * L;
      if (r < vr && c < vc) {
        const double v = (double)X[(int64_t)r * ld + c];
        const double p = v * v;
        x = xsum_add(xsum_add(x, p), __builtin_fma(v, v, -p));
      }
    }
    const XSum t = merge_x(x);
    if (tid == 0) {
      s_certified = (t.exact && isfinite(t.s)) ? 1 : 0;
      if (s_certified) s_sum = t.s + t.c;
    }
    __syncthreads();
  }
  if (!s_certified) {
    // Otherwise every square and its error go into an exact long accumulator
    // in LDS, and one thread rounds it once.
    __shared__ int64_t s_acc[kAccLimbs];
    for (int k = tid; k < kAccLimbs; k += kThreads) s_acc[k] = 0;
    __syncthreads();
    for (int e = tid; e < L * L; e += kThreads) {
      const int r = e / L, c = e - (e / L) * L;
      if (r < vr && c < vc) {
        const double x = (double)X[(int64_t)r * ld + c];
        const double p = x * x;
        lacc_add(s_acc, p);
        lacc_add(s_acc, __builtin_fma(x, x, -p));
      }
    }
    __syncthreads();
    if (tid == 0) s_sum = lacc_round(s_acc);
  }
  if (tid == 0) {
    const StatAcc &t = s_w[0];
    tdgemm_block_stats st;
    st.mn = t.mn;
    st.mx = t.mx;
    st.sumsq = s_sum;
    st.n = (int64_t)vr * vc;
    *out = st;
  }
}

// Non-dominated points of the calibration grid, per W row (see argmin_nsr):
// point k is kept when s[k] is finite and s[k] / R[k] is below s[k'] / R[k']
// for every k' > k (R strictly ascending). One wavefront per row; lane q owns
// the points [8q, 8q + 8), suffix minima and the compaction run across lanes.
__device__ __forceinline__ void build_table(const double *__restrict__ r,
                                            const double *__restrict__ s, int n_r,
                                            PlanTable *tab) {
  constexpr int PER = kMaxR / kWave;
  const int q = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  if (q >= 3) return;
  double ratio[PER];
  double cmin = INFINITY;
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int k = lane * PER + m;
    ratio[m] = INFINITY;
    if (k < n_r) {
      const double sk = s[q * n_r + k];
      if (sk < INFINITY) ratio[m] = sk / r[k];
    }
    cmin = fmin(cmin, ratio[m]);
  }
  double suf = cmin;                                // min over lanes >= this one
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double o = __shfl_down(suf, off);
    if (lane + off < kWave) suf = fmin(suf, o);
  }
  double run = __shfl_down(suf, 1);                 // min over lanes > this one
  if (lane == kWave - 1) run = INFINITY;
  bool keep[PER];
  int c = 0;
#pragma unroll
  for (int m = PER - 1; m >= 0; --m) {
    keep[m] = ratio[m] < run;                       // also false for s = +inf
    run = fmin(run, ratio[m]);
    c += keep[m] ? 1 : 0;
  }
  int pre = c;                                      // inclusive prefix over lanes
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(pre, off);
    if (lane >= off) pre += o;
  }
  int pos = pre - c;
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    if (!keep[m]) continue;
    const int k = lane * PER + m;
    const double sk = s[q * n_r + k];
    tab->idx[q][pos] = (short)k;
    tab->fr[q][pos] = (float)(1.0 / r[k]);
    tab->fs2[q][pos] = (float)(sk * sk);
    ++pos;
  }
  if (lane == kWave - 1) tab->cnt[q] = pre;
}

// Grid: one workgroup per block of A, then one per block of B, then (SNR
// control) one that builds the calibration table.
template <typename T, int L>
__global__ __launch_bounds__(kThreads) void k_stats(StatsArgs a) {
  const int64_t nbA = a.nI * a.nL, nbB = a.nL * a.nJ;
  const int64_t b = blockIdx.x;
  if (b < nbA) {                                    // block (i, l) of A, M x K
    const int64_t i = b / a.nL, l = b - (b / a.nL) * a.nL;
    const int vm = (int)min<int64_t>(L, a.M - i * L), vk = (int)min<int64_t>(L, a.K - l * L);
    const T *X = static_cast<const T *>(a.A);
    if (a.ta) block_stats<T, L>(X + (l * L) * a.lda + i * L, a.lda, vk, vm, &a.stats_a[b]);
    else      block_stats<T, L>(X + (i * L) * a.lda + l * L, a.lda, vm, vk, &a.stats_a[b]);
  } else if (b < nbA + nbB) {                       // block (l, j) of B, K x N
    const int64_t bb = b - nbA;
    const int64_t l = bb / a.nJ, j = bb - (bb / a.nJ) * a.nJ;
    const int vk = (int)min<int64_t>(L, a.K - l * L), vn = (int)min<int64_t>(L, a.N - j * L);
    const T *X = static_cast<const T *>(a.B);
    if (a.tb) block_stats<T, L>(X + (j * L) * a.ldb + l * L, a.ldb, vn, vk, &a.stats_b[bb]);
    else      block_stats<T, L>(X + (l * L) * a.ldb + j * L, a.ldb, vk, vn, &a.stats_b[bb]);
  } else {
    build_table(a.calib_r, a.calib_s, a.n_r, a.table);
  }
}

// ---------------------------------------------------------------------------
// Plan: one wavefront per inner kernel (i, j); lane q handles l = q + 64 t (with
// 65 to 256 subblocks, one workgroup per inner kernel, see kWide below).
// For every allowed W > 1 it finds the option of Sec. 5.B (argmin of the eq. 27
// noise over the calibrated grid), then prunes top-down (Sec. 6): while the
// exactly rounded sum of the current D exceeds the budget, the pair with the
// largest D (lowest l on ties) drops to the next smaller allowed W.
//
// When every pair's D strictly decreases from one allowed W to the next (the
// usual case), the greedy removes the "entries" (pair l at level v, value
// D_v(l) > 0) in the order of descending D, lowest l first among equals: an
// entry of l only becomes current once the larger entries of l are gone, and
// they come earlier in that order anyway. The sum after t removals is then
// non-increasing in t, and the greedy's stopping point -- the first t whose
// exactly rounded sum is within the budget -- is found by bisection over t
// from the entries' ranks. Under the throughput constraint the same order
// holds, and while no drop adds saved work the stopping point -- the last t
// that keeps the saving at the target -- is found the same way. Otherwise the
// greedy runs step by step.
constexpr int kMaxT = 8;          // up to 512 subblocks along K
constexpr int kMaxOpt = 4;        // allowed W levels: at most {4, 3, 2, 1} (L = 96)

struct PlanArgs {
  Problem pb;
  const tdgemm_block_stats *stats_a;   // [nI][nL]
  const tdgemm_block_stats *stats_b;   // [nL][nJ]
  tdgemm_pair *pairs;                  // [nI][nJ][nL]
  double *budget;                      // [nI][nJ]
  const double *calib_r;               // [n_r]
  const double *calib_s;               // [3][n_r]
  const PlanTable *table;
  int n_r;
  int ctrl;
  int n_opt;                           // allowed W levels, descending in w_desc
  int w_desc[kMaxOpt];
  int fixed_w;
  int block_scaled;                    // INT8 / FP8 form: separable records with W = 1
  double fixed_rmax, sep_q, u_safe;
  double snr_lin;                      // 10^(-S/10), computed on the host
  double accel;                        // F_kernel of the throughput constraint
  int units[5];                        // saved work per pair at packing W (units[1] = 0)
  const double *tile;                  // per-inner-kernel snr_lin / accel / tgt_pow, or nullptr
  double tgt_pow;                      // TARGET: 10^(S/10), computed on the host
};

__device__ __forceinline__ int srow(int W) { return W - 2; }   // s table row of W

// The largest d over the wavefront, the lowest l among equals, and the value w
// that comes with it; every lane gets the result. A maximum under this total
// order does not depend on the order of the merges, so the steps run as in
// wave_sum_exact (four DPP moves, two ds_bpermute exchanges). l = INT64_MAX
// marks a lane without a candidate. Every lane must be active.
template <int OFF>
__device__ __forceinline__ void argmax_step(double &d, int &l, int &w) {
  const double od = lane_partner<OFF>(d);
  const int ol = lane_partner<OFF>(l), ow = lane_partner<OFF>(w);
  if (od > d || (od == d && ol < l)) { d = od; l = ol; w = ow; }
}
__device__ __forceinline__ void wave_argmax(double &d, int64_t &l64, int &w) {
  int l = l64 == INT64_MAX ? INT_MAX : (int)l64;     // l < 2^31 (at most 512 subblocks)
  argmax_step<1>(d, l, w);
  argmax_step<2>(d, l, w);
  argmax_step<4>(d, l, w);
  argmax_step<8>(d, l, w);
  argmax_step<16>(d, l, w);
  argmax_step<32>(d, l, w);
  l64 = l == INT_MAX ? INT64_MAX : (int64_t)l;
}

// Lane k's value of v, for k uniform over the wavefront.
__device__ __forceinline__ int64_t lane_at(int64_t v, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), k);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Order key of a double that is not negative and not NaN: its bits with the
// sign cleared (so -0 keys as +0). Keys compare as integers exactly as the
// values compare as numbers, +inf included.
__device__ __forceinline__ int64_t order_key(double d) { return __double_as_longlong(d) & INT64_MAX; }

// Sum over the wavefront in plain double arithmetic (not exactly rounded; the
// value of lane 0 for every lane). Every lane must be active.
__device__ __forceinline__ double wave_sum_fast(double s) {
  s += lane_partner<1>(s);
  s += lane_partner<2>(s);
  s += lane_partner<4>(s);
  s += lane_partner<8>(s);
  s += lane_partner<16>(s);
  s += lane_partner<32>(s);
  return lane0(s);
}

// argmin_nsr (with LP = 1) for the TT subblocks of a lane at once; act[t]:
// subblock t exists and its pair has nonzero ranges. One pass over the table
// serves all of them, so their chains interleave; each result equals
// argmin_nsr's (the same FP32 threshold, then the first exact minimum in
// ascending order).
template <int TT>
__device__ __forceinline__ void argmin_nsr_lanes(const double (&L_eff)[TT], const BlockMoments (&a)[TT],
                                                 const BlockMoments (&b)[TT], const bool (&act)[TT],
                                                 const double *r, const double *s, const short *idx,
                                                 const float *fr, const float *fs2, int cnt, int (&kout)[TT]) {
  double ss[TT];
  float x0[TT], invL[TT], best[TT], thr[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    ss[t] = a[t].sigma * b[t].sigma;
    x0[t] = act[t] ? (float)(((L_eff[t] * a[t].amax) * b[t].amax) / ss[t]) : 0.0f;
    invL[t] = act[t] ? 1.0f / (float)L_eff[t] : 0.0f;
    best[t] = INFINITY;
  }
#pragma unroll 2
  for (int i = 0; i < cnt; ++i) {
    const float f = fr[i], g = fs2[i];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const float x = x0[t] * f;
      best[t] = fminf(best[t], x * ((1.0f / 6.0f) + x * ((1.0f / 144.0f) + g * invL[t])));
    }
  }
  int kbest[TT];
  double vbest[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    thr[t] = !act[t] ? -INFINITY : (best[t] < INFINITY) ? best[t] * (1.0f + 1e-5f) : INFINITY;
    kbest[t] = -1;
    vbest[t] = INFINITY;
  }
  for (int i = 0; i < cnt; ++i) {
    const float f = fr[i], g = fs2[i];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const float x = x0[t] * f;
      const float v = x * ((1.0f / 6.0f) + x * ((1.0f / 144.0f) + g * invL[t]));
      if (v <= thr[t]) {
        const int k = idx[i];
        const double e = nsr_exact(L_eff[t], a[t].amax, b[t].amax, ss[t], r[k], s[k]);
        if (e < vbest[t]) { vbest[t] = e; kbest[t] = k; }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TT; ++t) kout[t] = kbest[t];
}

// TT: subblocks per lane the kernel is compiled for (T = ceil(nL / 64) <= TT).
template <int TT>
__global__ __launch_bounds__(kThreads) void k_plan(PlanArgs a) {
  __shared__ float sh_fr[3][kMaxR], sh_fs2[3][kMaxR];
  __shared__ short sh_idx[3][kMaxR];
  __shared__ int sh_cnt[3];
  __shared__ double sh_scr[kThreads / kWave][kAccLimbs];
  // With two or four subblocks per lane a workgroup serves one inner kernel:
  // its first wavefront plans it, and all four count the ranks of the pruning
  // entries, a quarter of the slots each (the ranking is the longest chain).
  constexpr bool kWide = TT > 1 && TT < kMaxT;
  constexpr int kWaves = kThreads / kWave;
  constexpr int kEnt = (kMaxOpt - 1) * TT * kWave;
  __shared__ int64_t sh_keys[kWide ? kEnt : 1];
  __shared__ int sh_part[kWide ? kWaves - 1 : 1][kWide ? kEnt : 1];
  __shared__ int sh_need;
  // options over the calibrated grid: distortion (SNR) and throughput (ACCEL) control
  const bool snr = a.ctrl == TDGEMM_CTRL_SNR || a.ctrl == TDGEMM_CTRL_ACCEL;
  if (snr) {
    if (threadIdx.x < 3) sh_cnt[threadIdx.x] = a.table->cnt[threadIdx.x];
    for (int e = threadIdx.x; e < 3 * kMaxR; e += kThreads) {
      const int q = e / kMaxR, k = e - (e / kMaxR) * kMaxR;
      if (k < a.table->cnt[q]) {
        sh_idx[q][k] = a.table->idx[q][k];
        sh_fr[q][k] = a.table->fr[q][k];
        sh_fs2[q][k] = a.table->fs2[q][k];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int64_t tile = kWide ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * kWaves + wv;
  const Problem &pb = a.pb;
  if (tile >= pb.nI * pb.nJ) return;              // the whole workgroup when kWide
  const int64_t i = tile / pb.nJ, j = tile - (tile / pb.nJ) * pb.nJ;
  const int T = (int)((pb.nL + kWave - 1) / kWave);

  // per-(level, t) noise and chosen grid index, and current level per t
  double dopt[kMaxOpt][TT];
  int kopt[kMaxOpt][TT];
  int level[TT];
  double sigv[TT];                                // signal terms of the Sec. 6 budget
  // this wavefront's LDS for the long accumulator of an exact sum
  double *scr = sh_scr[threadIdx.x / kWave];
  // With one subblock per lane (nL <= 64), LP lanes share each subblock's
  // table scans (the plan is latency-bound and the scans are its longest
  // chains): subblock l is computed by lanes l LP .. l LP + LP - 1 and its
  // results are moved to lane l afterwards.
  int LP = 1;
  if (TT == 1)
    while (LP < 16 && 2 * LP * pb.nL <= kWave) LP *= 2;
  if (!kWide || wv == 0) {
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    level[t] = 0;
    sigv[t] = 0.0;
#pragma unroll
    for (int v = 0; v < kMaxOpt; ++v) { dopt[v][t] = 0.0; kopt[v][t] = -1; }
    if (t >= T) continue;
    const int64_t l = lane + (int64_t)kWave * t;
    if (l >= pb.nL) continue;
    const double L_eff = (double)min<int64_t>(pb.L, pb.K - l * pb.L);
    const BlockMoments ma = moments(a.stats_a[i * pb.nL + l]);
    const BlockMoments mb = moments(a.stats_b[l * pb.nJ + j]);
    sigv[t] = (L_eff * (ma.sigma * ma.sigma)) * (mb.sigma * mb.sigma);
  }
  if constexpr (TT != 1 && TT != kMaxT) {
    // several subblocks per lane: their table scans run together
    if (snr) {
      double Le[TT];
      BlockMoments ma[TT], mb[TT];
      bool act[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        act[t] = false;
        Le[t] = 1.0;
        ma[t] = BlockMoments{0.0, 1.0};
        mb[t] = BlockMoments{0.0, 1.0};
        const int64_t l = lane + (int64_t)kWave * t;
        if (t >= T || l >= pb.nL) continue;
        Le[t] = (double)min<int64_t>(pb.L, pb.K - l * pb.L);
        ma[t] = moments(a.stats_a[i * pb.nL + l]);
        mb[t] = moments(a.stats_b[l * pb.nJ + j]);
        act[t] = ma[t].amax != 0.0 && mb[t].amax != 0.0;   // else D = 0
      }
#pragma unroll 1
      for (int v = 0; v < a.n_opt; ++v) {
        const int W = a.w_desc[v];
        if (W == 1) continue;                     // D = 0
        const int q = srow(W);
        const double *s = a.calib_s + q * a.n_r;
        int k[TT];
        argmin_nsr_lanes<TT>(Le, ma, mb, act, a.calib_r, s, sh_idx[q], sh_fr[q], sh_fs2[q], sh_cnt[q], k);
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          if (!act[t]) continue;
          const double d = (k[t] < 0) ? kDUnavailable
                                      : option_at(W, Le[t], ma[t], mb[t], a.calib_r[k[t]], s[k[t]], a.u_safe).d;
#pragma unroll
          for (int u = 0; u < kMaxOpt; ++u)
            if (u == v) { dopt[u][t] = d; kopt[u][t] = k[t]; }
        }
      }
    }
  } else {
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t >= T) continue;
    const int64_t l = (TT == 1) ? lane / LP : lane + (int64_t)kWave * t;   // subblock of this lane
    const int sub = (TT == 1) ? (lane & (LP - 1)) : 0;
    double dg[kMaxOpt];
    int kg[kMaxOpt];
#pragma unroll
    for (int v = 0; v < kMaxOpt; ++v) { dg[v] = 0.0; kg[v] = -1; }
    if (l < pb.nL && snr) {
      const double L_eff = (double)min<int64_t>(pb.L, pb.K - l * pb.L);
      const BlockMoments ma = moments(a.stats_a[i * pb.nL + l]);
      const BlockMoments mb = moments(a.stats_b[l * pb.nJ + j]);
      if (ma.amax != 0.0 && mb.amax != 0.0) {     // else D = 0
#pragma unroll 1
        for (int v = 0; v < a.n_opt; ++v) {
          const int W = a.w_desc[v];
          if (W == 1) continue;                   // D = 0
          const int q = srow(W);
          const double *s = a.calib_s + q * a.n_r;
          const int k = argmin_nsr(L_eff, ma, mb, a.calib_r, s, sh_idx[q], sh_fr[q], sh_fs2[q], sh_cnt[q],
                                   sub, LP);
          const double d = (k < 0) ? kDUnavailable
                                   : option_at(W, L_eff, ma, mb, a.calib_r[k], s[k], a.u_safe).d;
#pragma unroll
          for (int u = 0; u < kMaxOpt; ++u)
            if (u == v) { dg[u] = d; kg[u] = k; }
        }
      }
    }
    const bool own = lane + (int64_t)kWave * t < pb.nL;
#pragma unroll
    for (int v = 0; v < kMaxOpt; ++v) {
      const double dv = (TT == 1) ? __shfl(dg[v], lane * LP) : dg[v];
      const int kv = (TT == 1) ? __shfl(kg[v], lane * LP) : kg[v];
      dopt[v][t] = own ? dv : 0.0;
      kopt[v][t] = own ? kv : -1;
    }
  }
  }
  }

  // level of slot t after removing every entry ranked below `cut`
  auto total_at = [&](const int (&rank)[kMaxOpt - 1][TT], int cut) {
    double dvs[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      int lv = 0;
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v) lv += (rank[v][t] < cut) ? 1 : 0;
      dvs[t] = 0.0;
#pragma unroll
      for (int v = 0; v < kMaxOpt; ++v) if (lv == v) dvs[t] = dopt[v][t];
    }
    return wave_sum_exact<TT>(dvs, scr);
  };
  auto total_fast = [&](const int (&rank)[kMaxOpt - 1][TT], int cut) {
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      int lv = 0;
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v) lv += (rank[v][t] < cut) ? 1 : 0;
#pragma unroll
      for (int v = 0; v < kMaxOpt; ++v) if (lv == v) sum += dopt[v][t];
    }
    return wave_sum_fast(sum);
  };

  double budget = 0.0;
  const int n_ent = a.n_opt - 1;                  // entry levels 0 .. n_opt - 2

  // does every pair's D decrease strictly along its entries (and weakly to the floor)?
  auto monotone = [&]() {
    bool mono = true;
#pragma unroll
    for (int t = 0; t < TT; ++t)
#pragma unroll
      for (int v = 0; v + 1 < kMaxOpt; ++v) {
        if (v + 1 >= a.n_opt) continue;
        const double d0 = dopt[v][t], d1 = dopt[v + 1][t];
        if (!(d1 <= d0)) mono = false;
        if (v + 1 < n_ent && d1 > 0.0 && !(d0 > d1)) mono = false;
      }
    return __all(mono) != 0;
  };

  // Rank of each own entry with D > 0 among the entries of the inner kernel:
  // the entries with a larger D, or an equal D and a lower l (only entries with
  // D > 0 can be counted). The count runs over the n_ent levels in use, compiled
  // for each count, and over the subblocks that exist (lanes beyond nL hold
  // D = 0, which counts for no ranked entry), reading each entry from its lane.
  // Entries that are not ranked get INT_MAX. n_pos: ranked entries; n_unav:
  // those with D >= kDUnavailable, which rank first. Called only when the
  // entries are monotone, hence not negative and not NaN (order_key).
  int rank[kMaxOpt - 1][TT];
  int n_pos = 0, n_unav = 0;
  auto rank_entries = [&]() {
    auto count_above = [&](auto nec) {
      constexpr int NE = decltype(nec)::value;
      // entry e counts slot s when key_s > key_e - [l_s < l_e], i.e. when
      // key_e - key_s - [l_s < l_e] is negative: integer arithmetic only
      int64_t ke[NE][TT];
      int cnt[NE][TT];
#pragma unroll
      for (int v = 0; v < NE; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) { ke[v][t] = order_key(dopt[v][t]); cnt[v][t] = 0; }
#pragma unroll
      for (int vs = 0; vs < NE; ++vs)
#pragma unroll
        for (int ts = 0; ts < TT; ++ts) {
          if (ts >= T) continue;
          const int nk = (int)min<int64_t>(kWave, pb.nL - (int64_t)ts * kWave);
          const int64_t src = ke[vs][ts];
          // slots k .. k + Q - 1 at a time: independent chains for the single
          // wavefront of the SIMD
          auto count_slots = [&](int k, auto qc) {
            constexpr int Q = decltype(qc)::value;
            int64_t ks[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) ks[q] = lane_at(src, k + q);   // entry (vs, subblock ts 64 + k + q)
#pragma unroll
            for (int t = 0; t < TT; ++t)
#pragma unroll
              for (int v = 0; v < NE; ++v) {
                int c = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                  const int64_t lower = (int64_t)((uint32_t)(ts * kWave + k + q - (t * kWave + lane)) >> 31);
                  c += (int)((uint64_t)(ke[v][t] - ks[q] - lower) >> 63);
                }
                cnt[v][t] += c;
              }
          };
          int k = 0;
#pragma unroll 1
          for (; k + 4 <= nk; k += 4) count_slots(k, std::integral_constant<int, 4>{});
#pragma unroll 1
          for (; k < nk; ++k) count_slots(k, std::integral_constant<int, 1>{});
        }
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          int c = 0;
#pragma unroll
          for (int u = 0; u < NE; ++u) if (u == v) c = cnt[u][t];
          rank[v][t] = (v < n_ent && dopt[v][t] > 0.0) ? c : INT_MAX;
        }
    };
    if (n_ent == 1)      count_above(std::integral_constant<int, 1>{});
    else if (n_ent == 2) count_above(std::integral_constant<int, 2>{});
    else                 count_above(std::integral_constant<int, 3>{});
#pragma unroll
    for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        n_pos += __popcll(__ballot(rank[v][t] != INT_MAX));
        n_unav += __popcll(__ballot(rank[v][t] != INT_MAX && dopt[v][t] >= kDUnavailable));
      }
  };
  // levels after dropping every entry ranked below `cut` (INT_MAX: all)
  auto levels_at = [&](int cut) {
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      int lv = 0;
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v)
        lv += (v < n_ent && (cut == INT_MAX || rank[v][t] < cut)) ? 1 : 0;
      level[t] = lv;
    }
  };

  // Does the pruning below rank its entries? D must fall along every pair's
  // entries and, under the throughput constraint, no drop may add saved work.
  bool need_rank = false;
  if (!kWide || wv == 0) {
    bool gains = false;
#pragma unroll
    for (int v = 0; v + 1 < kMaxOpt; ++v)
      if (v < n_ent && a.units[a.w_desc[v]] < a.units[a.w_desc[v + 1]]) gains = true;
    const bool ranked = a.ctrl == TDGEMM_CTRL_SNR || (a.ctrl == TDGEMM_CTRL_ACCEL && !gains);
    need_rank = n_ent > 0 && ranked && monotone();
  }
  if constexpr (kWide) {
    // The first wavefront's entries go to LDS (entry (v, t) of lane q at
    // (v T + t) 64 + q); wavefront w counts the slot groups g = v T + t with
    // g = w mod 4 for every entry, and the first wavefront adds the counts.
    if (wv == 0) {
      if (lane == 0) sh_need = need_rank ? 1 : 0;
      if (need_rank) {
#pragma unroll
        for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
          for (int t = 0; t < TT; ++t)
            if (v < n_ent && t < T) sh_keys[(v * T + t) * kWave + lane] = order_key(dopt[v][t]);
      }
    }
    __syncthreads();
    const bool counting = sh_need != 0;
    int cnt[kMaxOpt - 1][TT];
#pragma unroll
    for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
      for (int t = 0; t < TT; ++t) cnt[v][t] = 0;
    auto count_wide = [&](auto nec) {
      constexpr int NE = decltype(nec)::value;
      int64_t ke[NE][TT];
      int c[NE][TT];
#pragma unroll
      for (int v = 0; v < NE; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          ke[v][t] = t < T ? sh_keys[(v * T + t) * kWave + lane] : 0;
          c[v][t] = 0;
        }
#pragma unroll 1
      for (int g = wv; g < NE * T; g += kWaves) {
        const int ts = g % T;
        const int nk = (int)min<int64_t>(kWave, pb.nL - (int64_t)ts * kWave);
        const int64_t *slot = sh_keys + g * kWave;
        auto count_slots = [&](int k, auto qc) {
          constexpr int Q = decltype(qc)::value;
          int64_t ks[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) ks[q] = slot[k + q];
#pragma unroll
          for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int v = 0; v < NE; ++v) {
              int cc = 0;
#pragma unroll
              for (int q = 0; q < Q; ++q) {
                const int64_t lower = (int64_t)((uint32_t)(ts * kWave + k + q - (t * kWave + lane)) >> 31);
                cc += (int)((uint64_t)(ke[v][t] - ks[q] - lower) >> 63);
              }
              c[v][t] += cc;
            }
        };
        int k = 0;
#pragma unroll 1
        for (; k + 4 <= nk; k += 4) count_slots(k, std::integral_constant<int, 4>{});
#pragma unroll 1
        for (; k < nk; ++k) count_slots(k, std::integral_constant<int, 1>{});
      }
#pragma unroll
      for (int v = 0; v < NE; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) cnt[v][t] = c[v][t];
    };
    if (counting) {
      if (n_ent == 1)      count_wide(std::integral_constant<int, 1>{});
      else if (n_ent == 2) count_wide(std::integral_constant<int, 2>{});
      else                 count_wide(std::integral_constant<int, 3>{});
      if (wv > 0) {
#pragma unroll
        for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
          for (int t = 0; t < TT; ++t)
            if (v < n_ent && t < T) sh_part[wv - 1][(v * T + t) * kWave + lane] = cnt[v][t];
      }
    }
    __syncthreads();
    if (wv != 0) return;
    if (need_rank) {
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          int total = cnt[v][t];
          if (v < n_ent && t < T)
            for (int w = 0; w < kWaves - 1; ++w) total += sh_part[w][(v * T + t) * kWave + lane];
          rank[v][t] = (v < n_ent && dopt[v][t] > 0.0) ? total : INT_MAX;
        }
#pragma unroll
      for (int v = 0; v < kMaxOpt - 1; ++v)
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          n_pos += __popcll(__ballot(rank[v][t] != INT_MAX));
          n_unav += __popcll(__ballot(rank[v][t] != INT_MAX && dopt[v][t] >= kDUnavailable));
        }
    }
  } else {
    if (need_rank) rank_entries();
  }

  if (a.ctrl == TDGEMM_CTRL_ACCEL && n_ent > 0) {
    // Throughput constraint: the pair with the largest current D (lowest l among
    // equals) drops one level while the inner kernel keeps saving at least
    // accel * nL * units[W_max] and that D is positive. units[W] is the work a
    // pair saves at W in integers: twelfths of a W = 1 product, 12 - 12 / W, or
    // units of measured time from the accelerations F_W (Sec. 5.B). An
    // unavailable option (D >= kDUnavailable) drops whatever the constraint:
    // its product cannot be formed.
    int64_t own = 0;
#pragma unroll
    for (int t = 0; t < TT; ++t)
      if (t < T && lane + (int64_t)kWave * t < pb.nL) own += a.units[a.w_desc[0]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) own += __shfl_xor(own, off);
    const double frac = a.tile ? a.tile[i * pb.nJ + j] : a.accel;
    const double target = (frac * (double)pb.nL) * (double)a.units[a.w_desc[0]];
    if (need_rank) {
      // With D falling along every pair's entries, the greedy drops entries in
      // rank order; with no drop adding saved work, the saving only falls along
      // that order. The greedy therefore stops at the longest prefix of the
      // ranking that keeps the saving at or above the target (the unavailable
      // entries, ranked first, whatever it), found by bisection.
      auto saved_at = [&](int cut) {
        int64_t s = 0;
#pragma unroll
        for (int v = 0; v + 1 < kMaxOpt; ++v)
#pragma unroll
          for (int t = 0; t < TT; ++t)
            if (v < n_ent && rank[v][t] < cut) s += a.units[a.w_desc[v]] - a.units[a.w_desc[v + 1]];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        return own - s;
      };
      int lo = n_unav, hi = n_pos;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (!((double)saved_at(mid) < target)) lo = mid;   // the greedy's test, NaN included
        else hi = mid - 1;
      }
      levels_at(lo);
    } else {
      int64_t saved = own;
      for (;;) {
        double bd = -INFINITY;
        int64_t bl = INT64_MAX;
        int bdelta = 0;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const int64_t l = lane + (int64_t)kWave * t;
          if (t >= T || l >= pb.nL || level[t] >= a.n_opt - 1) continue;
          double dv = 0.0;
          int wc = 1, wn = 1;
#pragma unroll
          for (int v = 0; v < kMaxOpt; ++v)
            if (level[t] == v) { dv = dopt[v][t]; wc = a.w_desc[v]; wn = a.w_desc[v + 1 < kMaxOpt ? v + 1 : v]; }
          if (dv > bd || (dv == bd && l < bl)) { bd = dv; bl = l; bdelta = a.units[wc] - a.units[wn]; }
        }
        wave_argmax(bd, bl, bdelta);
        if (bl == INT64_MAX || !(bd > 0.0)) break;
        if (bd < kDUnavailable && (double)(saved - bdelta) < target) break;
        saved -= bdelta;
        if ((bl & (kWave - 1)) == lane) {
          const int tt = (int)(bl / kWave);
#pragma unroll
          for (int t = 0; t < TT; ++t) if (t == tt) level[t] += 1;
        }
      }
    }
  } else if (a.ctrl == TDGEMM_CTRL_SNR && n_ent > 0) {
    budget = (a.tile ? a.tile[i * pb.nJ + j] : a.snr_lin) * wave_sum_exact<TT>(sigv, scr);
    if (need_rank) {
      // the greedy's test for stopping: the sum does not exceed the budget (so
      // that a NaN budget stops it at once, as it stops the step-by-step greedy)
      auto within = [&](double total) { return !(total > budget); };
      int cut;
      if (!within(total_at(rank, n_pos))) {
        cut = INT_MAX;                            // the greedy empties every entry
      } else {
        // The exact total falls with the cut, so the cut is the smallest one
        // whose exact total is within the budget. A bisection over plain sums
        // proposes it, and two exact totals confirm it (the proposal within the
        // budget, its predecessor not); otherwise the bisection runs again over
        // exact totals.
        int lo = n_unav, hi = n_pos;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (within(total_fast(rank, mid))) hi = mid;
          else lo = mid + 1;
        }
        const bool found = (lo == n_pos || within(total_at(rank, lo))) &&
                           (lo == n_unav || !within(total_at(rank, lo - 1)));
        if (!found) {
          lo = n_unav;
          hi = n_pos;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (within(total_at(rank, mid))) hi = mid;
            else lo = mid + 1;
          }
        }
        cut = lo;
      }
      levels_at(cut);
    } else {
      for (;;) {
        double dvs[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          dvs[t] = 0.0;
#pragma unroll
          for (int v = 0; v < kMaxOpt; ++v) if (level[t] == v) dvs[t] = dopt[v][t];
        }
        const double total = wave_sum_exact<TT>(dvs, scr);
        // candidate with the largest current D, lowest l among equals
        double bd = -INFINITY;
        int64_t bl = INT64_MAX;
#pragma unroll
        for (int t = 0; t < TT; ++t) {
          const int64_t l = lane + (int64_t)kWave * t;
          if (t >= T || l >= pb.nL || level[t] >= a.n_opt - 1) continue;
          double dv = 0.0;
#pragma unroll
          for (int v = 0; v < kMaxOpt; ++v) if (level[t] == v) dv = dopt[v][t];
          if (dv > bd || (dv == bd && l < bl)) { bd = dv; bl = l; }
        }
        int unused = 0;
        wave_argmax(bd, bl, unused);
        if (bl == INT64_MAX) break;               // everything already at the lowest W
        // within the budget, and no unavailable option left (they are the largest D)
        if (!(total > budget) && bd < kDUnavailable) break;
        if ((bl & (kWave - 1)) == lane) {
          const int tt = (int)(bl / kWave);
#pragma unroll
          for (int t = 0; t < TT; ++t) if (t == tt) level[t] += 1;
        }
      }
    }
  } else if (a.ctrl == TDGEMM_CTRL_SNR) {
    budget = (a.tile ? a.tile[i * pb.nJ + j] : a.snr_lin) * wave_sum_exact<TT>(sigv, scr);
  }

  // Prop. 3 control: s(R_max, W) at the smallest grid R not below R_max (+inf
  // beyond the grid), by bisection over the ascending R values
  double s_target = 0.0;
  if (a.ctrl == TDGEMM_CTRL_TARGET && a.fixed_w > 1) {
    int lo = 0, hi = a.n_r;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (a.calib_r[mid] < a.fixed_rmax) lo = mid + 1; else hi = mid;
    }
    s_target = lo < a.n_r ? a.calib_s[srow(a.fixed_w) * a.n_r + lo] : INFINITY;
  }

  // final records
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t >= T) continue;
    const int64_t l = lane + (int64_t)kWave * t;
    if (l >= pb.nL) continue;
    const double L_eff = (double)min<int64_t>(pb.L, pb.K - l * pb.L);
    const BlockMoments ma = moments(a.stats_a[i * pb.nL + l]);
    const BlockMoments mb = moments(a.stats_b[l * pb.nJ + j]);
    const bool zero = (ma.amax == 0.0 || mb.amax == 0.0);
    tdgemm_pair o;
    if (snr) {
      int v = 0, k = -1;
#pragma unroll
      for (int q = 0; q < kMaxOpt; ++q) if (level[t] == q) { v = q; k = kopt[q][t]; }
      const int W = a.w_desc[v];
      if (W == 1) o = option_native();
      else if (zero) o = option_zero(W, a.u_safe);
      else if (k < 0) { o = option_zero(W, a.u_safe); o.d = kDUnavailable; o.s_rep = INFINITY; }
      else o = option_at(W, L_eff, ma, mb, a.calib_r[k], a.calib_s[srow(W) * a.n_r + k], a.u_safe);
    } else if (a.block_scaled) {
      o = zero ? option_zero(1, a.u_safe) : option_separable(1, L_eff, ma, mb, a.sep_q, a.u_safe);
    } else {
      const int W = a.fixed_w;
      if (W == 1) o = option_native();
      else if (zero) o = option_zero(W, a.u_safe);
      else if (a.ctrl == TDGEMM_CTRL_FIXED) o = option_at(W, L_eff, ma, mb, a.fixed_rmax, 0.0, a.u_safe);
      else if (a.ctrl == TDGEMM_CTRL_TARGET)
        o = option_target(W, L_eff, ma, mb, a.fixed_rmax, s_target,
                          a.tile ? a.tile[i * pb.nJ + j] : a.tgt_pow, a.u_safe);
      else o = option_separable(W, L_eff, ma, mb, a.sep_q, a.u_safe);
    }
    a.pairs[(i * pb.nJ + j) * pb.nL + l] = o;
  }
  if (lane == 0) a.budget[i * pb.nJ + j] = budget;
}

// ---------------------------------------------------------------------------
template <typename T, int L>
static void launch_stats_t(const StatsArgs &a, unsigned blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_stats<T, L>), dim3(blocks), dim3(kThreads), 0, st, a);
}

hipError_t launch_stats(const StatsArgs &a, int dtype, int L, hipStream_t st) {
  const int64_t blocks = a.nI * a.nL + a.nL * a.nJ + (a.table ? 1 : 0);
  if (blocks == 0) return hipSuccess;
  const unsigned nb = (unsigned)blocks;
  if (dtype == TDGEMM_F64) {
    if (L == 64)      launch_stats_t<double, 64>(a, nb, st);
    else if (L == 96) launch_stats_t<double, 96>(a, nb, st);
    else              launch_stats_t<double, 128>(a, nb, st);
  } else {
    if (L == 64)      launch_stats_t<float, 64>(a, nb, st);
    else if (L == 96) launch_stats_t<float, 96>(a, nb, st);
    else              launch_stats_t<float, 128>(a, nb, st);
  }
  return hipGetLastError();
}

hipError_t launch_plan(const PlanLaunch &p, hipStream_t st) {
  PlanArgs a;
  a.pb = p.pb;
  a.stats_a = p.stats_a;
  a.stats_b = p.stats_b;
  a.pairs = p.pairs;
  a.budget = p.budget;
  a.calib_r = p.calib_r;
  a.calib_s = p.calib_s;
  a.table = p.table;
  a.n_r = p.n_r;
  a.ctrl = p.ctrl;
  a.n_opt = p.n_opt;
  for (int v = 0; v < kMaxOpt; ++v) a.w_desc[v] = p.w_desc[v];
  a.fixed_w = p.fixed_w;
  a.block_scaled = p.block_scaled;
  a.fixed_rmax = p.fixed_rmax;
  a.sep_q = p.sep_q;
  a.u_safe = p.u_safe;
  a.snr_lin = p.snr_lin;
  a.accel = p.accel;
  for (int w = 0; w < 5; ++w) a.units[w] = p.units[w];
  a.tile = p.tile;
  a.tgt_pow = p.tgt_pow;
  const int64_t tiles = p.pb.nI * p.pb.nJ;
  const unsigned blocks = (unsigned)((tiles + (kThreads / kWave) - 1) / (kThreads / kWave));
  const int64_t T = (p.pb.nL + kWave - 1) / kWave;
  if (T <= 1)      hipLaunchKernelGGL(k_plan<1>, dim3(blocks), dim3(kThreads), 0, st, a);
  else if (T <= 2) hipLaunchKernelGGL(k_plan<2>, dim3((unsigned)tiles), dim3(kThreads), 0, st, a);   // one inner kernel per workgroup
  else if (T <= 4) hipLaunchKernelGGL(k_plan<4>, dim3((unsigned)tiles), dim3(kThreads), 0, st, a);
  else             hipLaunchKernelGGL(k_plan<kMaxT>, dim3(blocks), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace tdg
