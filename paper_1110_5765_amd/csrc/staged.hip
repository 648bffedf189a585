// Staged path: one kernel per step of Sec. 3, every intermediate in device
// memory, one L x L slot of `prec` elements per subblock pair.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace tdg {

template <typename T>
__device__ __forceinline__ double load_elem(const T *X, int64_t r, int64_t c, int64_t rows,
                                            int64_t cols, int64_t ld, bool tr) {
  if (r >= rows || c >= cols) return 0.0;
  return tr ? (double)X[c * ld + r] : (double)X[r * ld + c];
}

__device__ __forceinline__ void pair_ijl(int64_t pair, const Problem &pb, int64_t &i, int64_t &j,
                                         int64_t &l) {
  l = pair % pb.nL;
  const int64_t ij = pair / pb.nL;
  j = ij % pb.nJ;
  i = ij / pb.nJ;
}

// Eq. (3) in the packing precision PT; W = 1 pairs pass the block through.
template <typename PT>
__device__ __forceinline__ PT compand_one(double x, double c, int W) {
  if (W == 1) return (PT)x;
  return rint((PT)c * (PT)x);
}

// ---------------------------------------------------------------------------
template <typename IT, typename PT>
__global__ __launch_bounds__(kThreads) void k_compand(GemmOperands g, const IT *A, const IT *B,
                                                      PT *qA, PT *qB) {
  const Problem &pb = g.pb;
  const int64_t pair = blockIdx.x;
  int64_t i, j, l;
  pair_ijl(pair, pb, i, j, l);
  const tdgemm_pair o = g.pairs[pair];
  const int L = pb.L;
  PT *oa = qA + pair * L * L;
  PT *ob = qB + pair * L * L;
  for (int e = threadIdx.x; e < L * L; e += kThreads) {
    const int m = e / L, k = e - (e / L) * L;
    oa[e] = compand_one<PT>(load_elem(A, i * L + m, l * L + k, pb.M, pb.K, pb.lda, g.ta), o.c_a, o.w);
    ob[e] = compand_one<PT>(load_elem(B, l * L + m, j * L + k, pb.K, pb.N, pb.ldb, g.tb), o.c_b, o.w);
  }
}

// Eqs. (6), (7), (11): Horner's rule from the highest slot, acc = acc * z + q_i.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_pack(GemmOperands g, const PT *qA, const PT *qB,
                                                   PT *pA, PT *pB) {
  const int64_t pair = blockIdx.x;
  const tdgemm_pair o = g.pairs[pair];
  const int L = g.pb.L, W = o.w;
  const PT z = (PT)ldexp(1.0, -o.p), zi = (PT)ldexp(1.0, o.p);
  const PT *qa = qA + pair * L * L;
  const PT *qb = qB + pair * L * L;
  PT *pa = pA + pair * L * L;
  PT *pb = pB + pair * L * L;
  const int Lw = L / W;
  if (g.form == TDGEMM_SYM) {
    for (int e = threadIdx.x; e < L * Lw; e += kThreads) {
      const int m = e / Lw, kb = e - (e / Lw) * Lw;          // pA: L x L/W
      PT acc = qa[m * L + W * kb + (W - 1)];
      for (int s = W - 2; s >= 0; --s) acc = acc * z + qa[m * L + W * kb + s];
      pa[e] = acc;
    }
    for (int e = threadIdx.x; e < Lw * L; e += kThreads) {
      const int kb = e / L, n = e - (e / L) * L;             // pB: L/W x L
      PT acc = qb[(W * kb + (W - 1)) * L + n];
      for (int s = W - 2; s >= 0; --s) acc = acc * zi + qb[(W * kb + s) * L + n];
      pb[e] = acc;
    }
  } else {
    for (int e = threadIdx.x; e < Lw * L; e += kThreads) {
      const int mb = e / L, k = e - (e / L) * L;             // pA: L/W x L
      PT acc = qa[(W * mb + (W - 1)) * L + k];
      for (int s = W - 2; s >= 0; --s) acc = acc * z + qa[(W * mb + s) * L + k];
      pa[e] = acc;
    }
    for (int e = threadIdx.x; e < L * L; e += kThreads) pb[e] = qb[e];
  }
}

// Eqs. (8) / (12): Rbar = pA pB per pair on the matrix cores. Each wave takes
// 16 x 16 output blocks in turn; every block is one MFMA chain over the packed
// index in ascending order, starting from 0.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_packed_product(GemmOperands g, const PT *pA,
                                                             const PT *pB, PT *Rbar) {
  const int64_t pair = blockIdx.x;
  const tdgemm_pair o = g.pairs[pair];
  const int L = g.pb.L, W = o.w;
  const bool sym = (g.form == TDGEMM_SYM) || W == 1;
  const int rows = sym ? L : L / W;       // output rows
  const int kd = sym ? L / W : L;         // packed inner extent
  const PT *pa = pA + pair * L * L;
  const PT *pb = pB + pair * L * L;
  PT *out = Rbar + pair * L * L;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  // row blocks of 16 (the last one partial when L / W is not a multiple of 16:
  // asymmetric W = 4 at L = 96); rows past the packed ones read 0 and are not written
  const int nrb = (rows + 15) / 16, ncb = L / 16;
  for (int blk = wave; blk < nrb * ncb; blk += kThreads / kWave) {
    const int rb = blk / ncb, cb = blk - (blk / ncb) * ncb;
    const int arow = rb * 16 + (lane & 15);
    typename Mfma<PT>::Acc acc = Mfma<PT>::zero();
    for (int ks = 0; ks < kd / 4; ++ks) {
      const PT av = arow < rows ? pa[arow * kd + ks * 4 + (lane >> 4)] : (PT)0;
      const PT bv = pb[(ks * 4 + (lane >> 4)) * L + cb * 16 + (lane & 15)];
      acc = Mfma<PT>::mma(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rb * 16 + Mfma<PT>::row(lane, r);
      if (row < rows) out[row * L + cb * 16 + (lane & 15)] = acc[r];
    }
  }
}

// Eqs. (9)-(10) / (13)-(14) for the element (m, n) of a pair's L x L result.
template <typename PT>
__device__ __forceinline__ PT unpack_one(const PT *rb, int m, int n, int L, const tdgemm_pair &o,
                                         int form) {
  if (o.w == 1) return rb[m * L + n];
  const PT z = (PT)ldexp(1.0, -o.p), zi = (PT)ldexp(1.0, o.p);
  if (form == TDGEMM_SYM) {
    const PT u = rint(rb[m * L + n]);
    return u - zi * rint(z * u);
  }
  const int W = o.w, mb = m / W, slot = m - (m / W) * W;
  PT t = rb[mb * L + n];
  PT r = rint(t);
  for (int s = 1; s <= slot; ++s) {
    t = zi * (t - r);
    r = rint(t);
  }
  return r;
}

template <typename PT>
__global__ __launch_bounds__(kThreads) void k_unpack_pairs(GemmOperands g, const PT *Rbar,
                                                           PT *r_int) {
  const int64_t pair = blockIdx.x;
  const tdgemm_pair o = g.pairs[pair];
  const int L = g.pb.L;
  const PT *rb = Rbar + pair * L * L;
  PT *out = r_int + pair * L * L;
  for (int e = threadIdx.x; e < L * L; e += kThreads) {
    const int m = e / L, n = e - (e / L) * L;
    out[e] = unpack_one<PT>(rb, m, n, L, o, g.form);
  }
}

// Eq. (5) and the l-sum of eq. (2): C = fma(r_l, inv_l, C), l ascending (one
// rounding per pair; W = 1 pairs add their native product), in groups of gsize
// consecutive l (each from zero), the group sums added in ascending order to zero.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_decompand_sum(GemmOperands g, const PT *Rbar, PT *C) {
  const Problem &pb = g.pb;
  const int L = pb.L;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t total = pb.nI * pb.nJ * L * L;
  if (e >= total) return;
  const int64_t tile = e / (L * L);
  const int mn = (int)(e - tile * L * L);
  const int m = mn / L, n = mn - (mn / L) * L;
  const int64_t i = tile / pb.nJ, j = tile - (tile / pb.nJ) * pb.nJ;
  const int64_t row = i * L + m, col = j * L + n;
  if (row >= pb.M || col >= pb.N) return;
  PT sum = (PT)0, acc = (PT)0;
  for (int64_t l = 0; l < pb.nL; ++l) {
    const int64_t pair = (i * pb.nJ + j) * pb.nL + l;
    const tdgemm_pair o = g.pairs[pair];
    const PT r = unpack_one<PT>(Rbar + pair * L * L, m, n, L, o, g.form);
    acc = (o.w == 1) ? acc + r : __builtin_fma(r, (PT)o.inv, acc);
    if ((l + 1) % g.gsize == 0 || l + 1 == pb.nL) {
      sum = sum + acc;
      acc = (PT)0;
    }
  }
  C[row * pb.ldc + col] = sum;
}

// C = 0 (an empty inner dimension).
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_fill_zero(PT *C, int64_t M, int64_t N, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= M * N) return;
  const int64_t r = e / N;
  C[r * ldc + (e - r * N)] = (PT)0;
}

// ---------------------------------------------------------------------------
// Calibration helpers.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_int_inputs(const double *u, int64_t n, double q,
                                                         PT *out) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e < n) out[e] = (PT)(floor(u[e] * (2.0 * q + 1.0)) - q);
}

// out2 = {sum e, sum e^2, count of non-finite e} with e = r - ref, compensated sums.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_error_moments(const PT *r, const double *ref,
                                                            int64_t n, double *out2) {
  CSum s1{0.0, 0.0}, s2{0.0, 0.0};
  double bad = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += kThreads) {
    const double d = (double)r[e] - ref[e];
    if (!(fabs(d) < INFINITY)) { bad += 1.0; continue; }
    s1 = csum_add(s1, d);
    s2 = csum_add(s2, d * d);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s1 = csum_merge(s1, CSum{__shfl_xor(s1.s, off), __shfl_xor(s1.c, off)});
    s2 = csum_merge(s2, CSum{__shfl_xor(s2.s, off), __shfl_xor(s2.c, off)});
    bad += __shfl_xor(bad, off);
  }
  __shared__ double sh[kThreads / kWave][5];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[w][0] = s1.s; sh[w][1] = s1.c; sh[w][2] = s2.s; sh[w][3] = s2.c; sh[w][4] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CSum t1{sh[0][0], sh[0][1]}, t2{sh[0][2], sh[0][3]};
    double tb = sh[0][4];
    for (int q = 1; q < kThreads / kWave; ++q) {
      t1 = csum_merge(t1, CSum{sh[q][0], sh[q][1]});
      t2 = csum_merge(t2, CSum{sh[q][2], sh[q][3]});
      tb += sh[q][4];
    }
    out2[0] = csum_value(t1);
    out2[1] = csum_value(t2);
    out2[2] = tb;
  }
}

// ---------------------------------------------------------------------------
// Launchers. Inputs of type IT feed packed precision PT: (f64, f64), (f32, f64)
// and (f32, f32) are instantiated.
#define TDG_DISPATCH_IN_PREC(g, BODY)                                  \
  do {                                                                 \
    if ((g).in_dtype == TDGEMM_F64 && (g).prec == TDGEMM_F64) {        \
      using IT = double; using PT = double; BODY;                      \
    } else if ((g).in_dtype == TDGEMM_F32 && (g).prec == TDGEMM_F64) { \
      using IT = float; using PT = double; BODY;                       \
    } else {                                                           \
      using IT = float; using PT = float; BODY;                        \
    }                                                                  \
  } while (0)

hipError_t launch_compand(const GemmOperands &g, const void *A, const void *B, void *qA, void *qB,
                          hipStream_t st) {
  TDG_DISPATCH_IN_PREC(g, hipLaunchKernelGGL((k_compand<IT, PT>), dim3((unsigned)g.pb.nI * g.pb.nJ * g.pb.nL),
                                             dim3(kThreads), 0, st, g, (const IT *)A, (const IT *)B,
                                             (PT *)qA, (PT *)qB));
  return hipGetLastError();
}

#define TDG_DISPATCH_PREC(prec, BODY)            \
  do {                                           \
    if ((prec) == TDGEMM_F64) { using PT = double; BODY; } \
    else { using PT = float; BODY; }             \
  } while (0)

static unsigned n_pair_blocks(const GemmOperands &g) {
  return (unsigned)(g.pb.nI * g.pb.nJ * g.pb.nL);
}

hipError_t launch_pack(const GemmOperands &g, const void *qA, const void *qB, void *pA, void *pB,
                       hipStream_t st) {
  TDG_DISPATCH_PREC(g.prec, hipLaunchKernelGGL((k_pack<PT>), dim3(n_pair_blocks(g)), dim3(kThreads),
                                               0, st, g, (const PT *)qA, (const PT *)qB, (PT *)pA,
                                               (PT *)pB));
  return hipGetLastError();
}

hipError_t launch_packed_product(const GemmOperands &g, const void *pA, const void *pB, void *Rbar,
                                 hipStream_t st) {
  TDG_DISPATCH_PREC(g.prec, hipLaunchKernelGGL((k_packed_product<PT>), dim3(n_pair_blocks(g)),
                                               dim3(kThreads), 0, st, g, (const PT *)pA,
                                               (const PT *)pB, (PT *)Rbar));
  return hipGetLastError();
}

hipError_t launch_unpack(const GemmOperands &g, const void *Rbar, void *r_int, void *C,
                         hipStream_t st) {
  if (r_int) {
    TDG_DISPATCH_PREC(g.prec, hipLaunchKernelGGL((k_unpack_pairs<PT>), dim3(n_pair_blocks(g)),
                                                 dim3(kThreads), 0, st, g, (const PT *)Rbar,
                                                 (PT *)r_int));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (C) {
    const int64_t total = g.pb.nI * g.pb.nJ * (int64_t)g.pb.L * g.pb.L;
    const unsigned blocks = (unsigned)((total + kThreads - 1) / kThreads);
    TDG_DISPATCH_PREC(g.prec, hipLaunchKernelGGL((k_decompand_sum<PT>), dim3(blocks), dim3(kThreads),
                                                 0, st, g, (const PT *)Rbar, (PT *)C));
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *C, int prec, int64_t M, int64_t N, int64_t ldc, hipStream_t st) {
  const unsigned blocks = (unsigned)((M * N + kThreads - 1) / kThreads);
  TDG_DISPATCH_PREC(prec, hipLaunchKernelGGL((k_fill_zero<PT>), dim3(blocks), dim3(kThreads), 0, st,
                                             (PT *)C, M, N, ldc));
  return hipGetLastError();
}

hipError_t launch_int_inputs(const double *u, int64_t n, double q, int prec, void *out,
                             hipStream_t st) {
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  TDG_DISPATCH_PREC(prec, hipLaunchKernelGGL((k_int_inputs<PT>), dim3(blocks), dim3(kThreads), 0, st,
                                             u, n, q, (PT *)out));
  return hipGetLastError();
}

hipError_t launch_error_moments(const void *r, const double *ref, int prec, int64_t n,
                                double *out2, hipStream_t st) {
  TDG_DISPATCH_PREC(prec, hipLaunchKernelGGL((k_error_moments<PT>), dim3(1), dim3(kThreads), 0, st,
                                             (const PT *)r, ref, n, out2));
  return hipGetLastError();
}

}  // namespace tdg
