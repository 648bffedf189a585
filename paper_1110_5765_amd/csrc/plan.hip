// Block statistics (Sec. 3, Sec. 5.B) and the per-pair plan with inner-kernel
// pruning (Sec. 5.B, Sec. 6).
#include "common.h"
#include "kernels.h"

namespace tdg {

// ---------------------------------------------------------------------------
// One workgroup per L x L block of a matrix X (rows x cols logically; stored
// transposed when TR). Threads stride through the block so that consecutive
// lanes read consecutive addresses: along a row when X is stored as given,
// along a column of the logical block when it is stored transposed.
// Writes min, max, the compensated sum of squares (TwoProduct via fma, TwoSum)
// and the number of valid elements.
template <typename T, bool TR>
__global__ __launch_bounds__(kThreads) void k_block_stats(const T *__restrict__ X, int64_t rows,
                                                          int64_t cols, int64_t ld, int L,
                                                          int64_t ncb, tdgemm_block_stats *out) {
  const int64_t rb = blockIdx.y, cb = blockIdx.x;
  const int64_t r0 = rb * L, c0 = cb * L;
  const int vr = (int)min<int64_t>(L, rows - r0);
  const int vc = (int)min<int64_t>(L, cols - c0);
  double mn = INFINITY, mx = -INFINITY;
  CSum acc{0.0, 0.0};
  const int n = L * L;
  for (int e = threadIdx.x; e < n; e += kThreads) {
    int r, c;
    if (!TR) { r = e / L; c = e - r * L; }
    else     { c = e / L; r = e - c * L; }
    if (r < vr && c < vc) {
      double x = TR ? (double)X[(c0 + c) * ld + (r0 + r)] : (double)X[(r0 + r) * ld + (c0 + c)];
      mn = fmin(mn, x);
      mx = fmax(mx, x);
      double p = x * x;
      double pe = __builtin_fma(x, x, -p);
      acc = csum_add(acc, p);
      acc.c = acc.c + pe;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off));
    mx = fmax(mx, __shfl_xor(mx, off));
    CSum y{__shfl_xor(acc.s, off), __shfl_xor(acc.c, off)};
    acc = csum_merge(acc, y);
  }
  __shared__ double s_mn[kThreads / kWave], s_mx[kThreads / kWave], s_s[kThreads / kWave],
      s_c[kThreads / kWave];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_mn[w] = mn; s_mx[w] = mx; s_s[w] = acc.s; s_c[w] = acc.c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CSum t{s_s[0], s_c[0]};
    double tmn = s_mn[0], tmx = s_mx[0];
    for (int q = 1; q < kThreads / kWave; ++q) {
      t = csum_merge(t, CSum{s_s[q], s_c[q]});
      tmn = fmin(tmn, s_mn[q]);
      tmx = fmax(tmx, s_mx[q]);
    }
    tdgemm_block_stats st;
    st.mn = tmn;
    st.mx = tmx;
    st.sumsq = csum_value(t);
    st.n = (int64_t)vr * vc;
    out[rb * ncb + cb] = st;
  }
}

// ---------------------------------------------------------------------------
// Plan: one wavefront per inner kernel (i, j); lane q handles l = q + 64 t.
// For every allowed W > 1 it finds the option of Sec. 5.B (argmin of the eq. 27
// noise over the calibrated grid), then prunes top-down (Sec. 6): while the
// exactly rounded sum of the current D exceeds the budget, the pair with the
// largest D (lowest l on ties) drops to the next smaller allowed W.
constexpr int kMaxT = 8;          // up to 512 subblocks along K
constexpr int kMaxR = 512;        // calibration grid points
constexpr int kMaxOpt = 3;        // allowed W levels: at most {4, 2, 1}

struct PlanArgs {
  Problem pb;
  const tdgemm_block_stats *stats_a;   // [nI][nL]
  const tdgemm_block_stats *stats_b;   // [nL][nJ]
  tdgemm_pair *pairs;                  // [nI][nJ][nL]
  double *budget;                      // [nI][nJ]
  const double *calib_r;               // [n_r]
  const double *calib_s;               // [3][n_r]
  int n_r;
  int ctrl;
  int n_opt;                           // allowed W levels, descending in w_desc
  int w_desc[kMaxOpt];
  int fixed_w;
  double fixed_rmax, sep_q, u_safe;
  double snr_lin;                      // 10^(-S/10), computed on the host
};

__device__ __forceinline__ int srow(int W) { return W - 2; }   // s table row of W

__global__ __launch_bounds__(kThreads) void k_plan(PlanArgs a) {
  __shared__ double sh_r[kMaxR], sh_s[3][kMaxR];
  __shared__ float sh_fr[3][kMaxR], sh_fs2[3][kMaxR];
  __shared__ short sh_idx[3][kMaxR];
  __shared__ unsigned char sh_keep[3][kMaxR];
  __shared__ int sh_cnt[3];
  const bool snr = a.ctrl == TDGEMM_CTRL_SNR;
  if (snr) {
    for (int k = threadIdx.x; k < a.n_r; k += kThreads) {
      sh_r[k] = a.calib_r[k];
      for (int q = 0; q < 3; ++q) sh_s[q][k] = a.calib_s[q * a.n_r + k];
    }
    __syncthreads();
    // non-dominated table points per W row (see argmin_nsr)
    for (int e = threadIdx.x; e < 3 * a.n_r; e += kThreads) {
      const int q = e / a.n_r, k = e - (e / a.n_r) * a.n_r;
      const double sk = sh_s[q][k];
      bool keep = sk < INFINITY;
      if (keep) {
        const double ratio = sk / sh_r[k];
        for (int k2 = k + 1; k2 < a.n_r && keep; ++k2) {
          const double s2 = sh_s[q][k2];
          if (s2 < INFINITY && sh_r[k2] > sh_r[k] && s2 / sh_r[k2] <= ratio) keep = false;
        }
      }
      sh_keep[q][k] = keep ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      const int q = threadIdx.x;
      int c = 0;
      for (int k = 0; k < a.n_r; ++k) {
        if (!sh_keep[q][k]) continue;
        sh_idx[q][c] = (short)k;
        sh_fr[q][c] = (float)(1.0 / sh_r[k]);
        sh_fs2[q][c] = (float)(sh_s[q][k] * sh_s[q][k]);
        ++c;
      }
      sh_cnt[q] = c;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t tile = (int64_t)blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
  const Problem &pb = a.pb;
  if (tile >= pb.nI * pb.nJ) return;
  const int64_t i = tile / pb.nJ, j = tile - (tile / pb.nJ) * pb.nJ;
  const int T = (int)((pb.nL + kWave - 1) / kWave);

  // per-(level, t) noise and chosen grid index, and current level per t
  double dopt[kMaxOpt][kMaxT];
  int kopt[kMaxOpt][kMaxT];
  int level[kMaxT];
  CSum sig{0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kMaxT; ++t) {
    level[t] = 0;
#pragma unroll
    for (int v = 0; v < kMaxOpt; ++v) { dopt[v][t] = 0.0; kopt[v][t] = -1; }
    if (t >= T) continue;
    const int64_t l = lane + (int64_t)kWave * t;
    if (l >= pb.nL) continue;
    const double L_eff = (double)min<int64_t>(pb.L, pb.K - l * pb.L);
    const BlockMoments ma = moments(a.stats_a[i * pb.nL + l]);
    const BlockMoments mb = moments(a.stats_b[l * pb.nJ + j]);
    sig = csum_add(sig, (L_eff * (ma.sigma * ma.sigma)) * (mb.sigma * mb.sigma));
    if (!snr) continue;
    const bool zero = (ma.amax == 0.0 || mb.amax == 0.0);
#pragma unroll
    for (int v = 0; v < kMaxOpt; ++v) {
      if (v >= a.n_opt) continue;
      const int W = a.w_desc[v];
      if (W == 1 || zero) continue;               // D = 0
      const int q = srow(W);
      const int k = argmin_nsr(L_eff, ma, mb, sh_r, sh_s[q], sh_idx[q], sh_fr[q], sh_fs2[q], sh_cnt[q]);
      kopt[v][t] = k;
      dopt[v][t] = (k < 0) ? kDUnavailable
                           : option_at(W, L_eff, ma, mb, sh_r[k], sh_s[srow(W)][k], a.u_safe).d;
    }
  }

  double budget = 0.0;
  if (snr) {
    budget = a.snr_lin * wave_csum(sig);
    for (;;) {
      CSum tot{0.0, 0.0};
#pragma unroll
      for (int t = 0; t < kMaxT; ++t) {
        double dv = 0.0;
#pragma unroll
        for (int v = 0; v < kMaxOpt; ++v) if (level[t] == v) dv = dopt[v][t];
        tot = csum_add(tot, dv);
      }
      const double total = wave_csum(tot);
      if (!(total > budget)) break;
      // candidate with the largest current D, lowest l among equals
      double bd = -INFINITY;
      int64_t bl = INT64_MAX;
#pragma unroll
      for (int t = 0; t < kMaxT; ++t) {
        const int64_t l = lane + (int64_t)kWave * t;
        if (t >= T || l >= pb.nL || level[t] >= a.n_opt - 1) continue;
        double dv = 0.0;
#pragma unroll
        for (int v = 0; v < kMaxOpt; ++v) if (level[t] == v) dv = dopt[v][t];
        if (dv > bd || (dv == bd && l < bl)) { bd = dv; bl = l; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        double od = __shfl_xor(bd, off);
        int64_t ol = __shfl_xor(bl, off);
        if (od > bd || (od == bd && ol < bl)) { bd = od; bl = ol; }
      }
      if (bl == INT64_MAX) break;                 // everything already at the lowest W
      if ((bl & (kWave - 1)) == lane) {
        const int tt = (int)(bl / kWave);
#pragma unroll
        for (int t = 0; t < kMaxT; ++t) if (t == tt) level[t] += 1;
      }
    }
  }

  // final records
#pragma unroll
  for (int t = 0; t < kMaxT; ++t) {
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
      else o = option_at(W, L_eff, ma, mb, sh_r[k], sh_s[srow(W)][k], a.u_safe);
    } else {
      const int W = a.fixed_w;
      if (W == 1) o = option_native();
      else if (zero) o = option_zero(W, a.u_safe);
      else if (a.ctrl == TDGEMM_CTRL_FIXED) o = option_at(W, L_eff, ma, mb, a.fixed_rmax, 0.0, a.u_safe);
      else o = option_separable(W, L_eff, ma, mb, a.sep_q, a.u_safe);
    }
    a.pairs[(i * pb.nJ + j) * pb.nL + l] = o;
  }
  if (lane == 0) a.budget[i * pb.nJ + j] = budget;
}

// ---------------------------------------------------------------------------
template <typename T>
static hipError_t launch_stats_t(const void *X, int64_t rows, int64_t cols, int64_t ld, bool tr,
                                 int L, tdgemm_block_stats *out, hipStream_t st) {
  const int64_t nrb = (rows + L - 1) / L, ncb = (cols + L - 1) / L;
  dim3 grid((unsigned)ncb, (unsigned)nrb);
  if (tr)
    hipLaunchKernelGGL((k_block_stats<T, true>), grid, dim3(kThreads), 0, st, (const T *)X, rows,
                       cols, ld, L, ncb, out);
  else
    hipLaunchKernelGGL((k_block_stats<T, false>), grid, dim3(kThreads), 0, st, (const T *)X, rows,
                       cols, ld, L, ncb, out);
  return hipGetLastError();
}

hipError_t launch_block_stats(const void *X, int dtype, int64_t rows, int64_t cols, int64_t ld,
                              bool tr, int L, tdgemm_block_stats *out, hipStream_t st) {
  return dtype == TDGEMM_F64 ? launch_stats_t<double>(X, rows, cols, ld, tr, L, out, st)
                             : launch_stats_t<float>(X, rows, cols, ld, tr, L, out, st);
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
  a.n_r = p.n_r;
  a.ctrl = p.ctrl;
  a.n_opt = p.n_opt;
  for (int v = 0; v < kMaxOpt; ++v) a.w_desc[v] = p.w_desc[v];
  a.fixed_w = p.fixed_w;
  a.fixed_rmax = p.fixed_rmax;
  a.sep_q = p.sep_q;
  a.u_safe = p.u_safe;
  a.snr_lin = p.snr_lin;
  const int64_t tiles = p.pb.nI * p.pb.nJ;
  const unsigned blocks = (unsigned)((tiles + (kThreads / kWave) - 1) / (kThreads / kWave));
  hipLaunchKernelGGL(k_plan, dim3(blocks), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace tdg
