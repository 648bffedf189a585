// Block-scaled INT8 / FP8 form (Remark 1) on the separable block scales
// c = Q / max|X| of Sec. 3.A: per-block quantization to byte operands, the
// per-pair products on the INT8 / FP8 matrix cores, and the float32 reverse
// companding and l-sum of eqs. (2), (5).
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace tdg {

constexpr int kL8 = 128;          // block size of the precision form
constexpr int kRow8 = kL8 + 16;   // LDS row stride in bytes (16-byte reads conflict-free)

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Quantization of one value to a byte.
// INT8: two's complement of [[c x]] (|c x| <= Q <= 127 by construction).
// E4M3: OCP E4M3FN code of the nearest value, ties to even mantissa, saturating
// at 448. For |v| >= 2^-6 with v in [2^e, 2^(e+1)), t = [[v 2^(3-e)]] lies in
// [8, 16] and the code is 8 e + 48 + t (t = 16 carries into the next binade);
// below 2^-6 the code is [[v 2^9]] (subnormals; 8 is the smallest normal).
// Both scalings are exact.
__device__ __forceinline__ uint8_t quant_i8(double v) { return (uint8_t)(int8_t)(int)rint(v); }

__device__ __forceinline__ uint8_t quant_e4m3(double v) {
  const uint8_t s = signbit(v) ? 0x80 : 0;
  const double a = fabs(v);
  int code;
  if (a < 0.015625) {
    code = (int)rint(a * 512.0);
  } else if (a >= 448.0) {
    code = 126;
  } else {
    const int e = ilogb(a);
    const int t = (int)rint(ldexp(a, 3 - e));
    code = min(8 * e + 48 + t, 126);
  }
  return s | (uint8_t)code;
}

template <int FMT>
__device__ __forceinline__ uint8_t quant8(double v) {
  return FMT == TDGEMM_I8 ? quant_i8(v) : quant_e4m3(v);
}

// ---------------------------------------------------------------------------
// One workgroup per block of A (i, l) or of B (l, j). The output tile is 128
// rows x 128 bytes with K contiguous: rows of A, or columns of B (B^T). The
// block is read in its stored layout (coalesced), quantized into an LDS tile
// in output layout, and written out in 16-byte rows.
template <typename T, int FMT>
__global__ __launch_bounds__(kThreads) void k_quant8(Quant8Args a) {
  __shared__ __align__(16) uint8_t tile[kL8][kRow8];
  const int64_t nbA = a.nI * a.nL;
  const int64_t b = blockIdx.x;
  const T *X;
  int64_t ld, r0, c0;                      // stored block origin
  int srows, scols;                        // valid stored extents
  bool direct;                             // stored rows are output rows
  const tdgemm_block_stats *st;
  uint8_t *out;
  if (b < nbA) {                           // A block (i, l): out rows m, K along columns
    const int64_t i = b / a.nL, l = b - (b / a.nL) * a.nL;
    const int vm = (int)min<int64_t>(kL8, a.M - i * kL8), vk = (int)min<int64_t>(kL8, a.K - l * kL8);
    X = static_cast<const T *>(a.A);
    ld = a.lda;
    direct = !a.ta;
    if (direct) { r0 = i * kL8; c0 = l * kL8; srows = vm; scols = vk; }
    else        { r0 = l * kL8; c0 = i * kL8; srows = vk; scols = vm; }
    st = &a.stats_a[b];
    out = a.qA + (i * kL8) * a.Kp + l * kL8;
  } else {                                 // B block (l, j): out rows n (B^T), K along columns
    const int64_t bb = b - nbA;
    const int64_t l = bb / a.nJ, j = bb - (bb / a.nJ) * a.nJ;
    const int vk = (int)min<int64_t>(kL8, a.K - l * kL8), vn = (int)min<int64_t>(kL8, a.N - j * kL8);
    X = static_cast<const T *>(a.B);
    ld = a.ldb;
    direct = a.tb;
    if (direct) { r0 = j * kL8; c0 = l * kL8; srows = vn; scols = vk; }
    else        { r0 = l * kL8; c0 = j * kL8; srows = vk; scols = vn; }
    st = &a.stats_b[bb];
    out = a.qB + (j * kL8) * a.Kp + l * kL8;
  }
  const BlockMoments mo = moments(*st);
  const double c = (mo.amax == 0.0) ? 0.0 : a.q / mo.amax;
  const T *base = X + r0 * ld + c0;
  const int tid = threadIdx.x;
  for (int e = tid; e < kL8 * kL8; e += kThreads) {
    const int sr = e / kL8, sc = e - (e / kL8) * kL8;
    uint8_t v = 0;
    if (sr < srows && sc < scols) v = quant8<FMT>(c * (double)base[(int64_t)sr * ld + sc]);
    if (direct) tile[sr][sc] = v;
    else        tile[sc][sr] = v;
  }
  __syncthreads();
  for (int e = tid; e < kL8 * (kL8 / 16); e += kThreads) {
    const int r = e / (kL8 / 16), ch = e - (e / (kL8 / 16)) * (kL8 / 16);
    *reinterpret_cast<v4i *>(out + (int64_t)r * a.Kp + ch * 16) =
        *reinterpret_cast<const v4i *>(&tile[r][ch * 16]);
  }
}

// ---------------------------------------------------------------------------
// Block-scaled product: one workgroup per inner kernel (i, j), a 128 x 128 tile
// of C; four wavefronts in 2 x 2, each 64 x 64 = 4 x 4 matrix-core tiles. Per
// subblock l the byte tiles of A_il and B_lj^T are staged in LDS (double
// buffered, next l prefetched in registers), multiplied on the matrix cores
// (INT8 16x16x64 with exact INT32 results; FP8 16x16x128 with FP32 results),
// and then either written out per pair (STAGED) or added to C as
// C = fma(float(r), float(inv), C), l ascending.
// At most 256 registers per lane, so that two workgroups (64 KB of LDS each)
// share a CU and one's LDS waits and epilogue overlap the other's MFMAs.
//
// LDS rows are 128 bytes; the 16-byte chunk c of row r sits at chunk position
// c ^ ((r >> 1) & 7). Sixteen lanes reading (or writing) 16 bytes each from
// sixteen consecutive rows, or from two rows, then touch all 64 banks once.
__device__ __forceinline__ int swz8(int r, int c16) { return (c16 ^ ((r >> 1) & 7)) * 16; }

template <int FMT, bool STAGED>
__global__ __launch_bounds__(kThreads, 2) void k_gemm8(Gemm8Args a) {
  __shared__ __align__(16) uint8_t sa[2][kL8][kL8];
  __shared__ __align__(16) uint8_t sb[2][kL8][kL8];
  // XCD-aware order: workgroup b runs on XCD b mod 8; each XCD takes a
  // contiguous range of tiles, four tile rows at a time, so that its concurrent
  // workgroups share A and B panels in its L2 (5 % faster at 8192^3 than the
  // row-major order, which spread every A panel over all eight L2s)
  const int64_t ntl = a.nI * a.nJ, per = (ntl + 7) / 8;
  const int64_t lin = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lin >= ntl) return;
  const int64_t grp = lin / (4 * a.nJ), first_i = grp * 4;
  const int64_t gsz = min((int64_t)4, a.nI - first_i), in_grp = lin - grp * 4 * a.nJ;
  const int64_t i = first_i + in_grp % gsz, j = in_grp / gsz;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 4, li = lane & 15;
  const uint8_t *gA = a.qA + (i * kL8) * a.Kp;
  const uint8_t *gB = a.qB + (j * kL8) * a.Kp;

  // Raw buffer loads: the operand panels as buffer resources, each thread's
  // 16-byte chunks at fixed 32-bit offsets (r Kp + 16 c16 < 2^24, as Kp <= 2^16)
  // and the subblock l as a scalar offset, so the loop computes no addresses.
  v4i stage[8];                            // 4 chunks of A, 4 of B (16 bytes each)
  int goff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ch = tid + kThreads * q, r = ch >> 3, c16 = ch & 7;
    goff[q] = (int)(r * a.Kp + c16 * 16);
  }
  const int span = (int)(kL8 * a.Kp);      // bytes of one 128-row panel
  const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc((void *)gA, (short)0, span, kBufWord3);
  const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc((void *)gB, (short)0, span, kBufWord3);
  auto gload = [&](int64_t l) {
    const int so = (int)(l * kL8);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      stage[q] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rA, goff[q], so, 0));
      stage[4 + q] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(rB, goff[q], so, 0));
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = tid + kThreads * q, r = ch >> 3, c16 = ch & 7;
      *reinterpret_cast<v4i *>(&sa[buf][r][swz8(r, c16)]) = stage[q];
      *reinterpret_cast<v4i *>(&sb[buf][r][swz8(r, c16)]) = stage[4 + q];
    }
  };

  typedef typename std::conditional<FMT == TDGEMM_I8, v4i, v4f>::type acc_t;
  acc_t acc[4][4];
  v4f cacc[4][4];
  const acc_t zero = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) cacc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};

  // The products of pair l into acc: fragments of A, then per 32-column half h
  // of the wavefront's tile (y in {2h, 2h + 1}) the fragments of B and the MFMAs.
  typedef typename std::conditional<FMT == TDGEMM_I8, v4i, v8i>::type frag_t;
  constexpr int NKS = FMT == TDGEMM_I8 ? 2 : 1;           // k-steps per pair
  frag_t fa[NKS][4];
  auto read_a = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int r = wr * 64 + x * 16 + li;
        if constexpr (FMT == TDGEMM_I8) {
          fa[ks][x] = *reinterpret_cast<const v4i *>(&sa[buf][r][swz8(r, ks * 4 + g)]);
        } else {
          const v4i lo = *reinterpret_cast<const v4i *>(&sa[buf][r][swz8(r, 2 * g)]);
          const v4i hi = *reinterpret_cast<const v4i *>(&sa[buf][r][swz8(r, 2 * g + 1)]);
          fa[ks][x] = v8i{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
      }
  };
  auto mma_half = [&](int buf, auto hc) {
    constexpr int h = decltype(hc)::value;
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      frag_t fb[2];
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        const int r = wc * 64 + (2 * h + yy) * 16 + li;
        if constexpr (FMT == TDGEMM_I8) {
          fb[yy] = *reinterpret_cast<const v4i *>(&sb[buf][r][swz8(r, ks * 4 + g)]);
        } else {
          const v4i lo = *reinterpret_cast<const v4i *>(&sb[buf][r][swz8(r, 2 * g)]);
          const v4i hi = *reinterpret_cast<const v4i *>(&sb[buf][r][swz8(r, 2 * g + 1)]);
          fb[yy] = v8i{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int yy = 0; yy < 2; ++yy) {
          const int y = 2 * h + yy;
          // each pair's product starts from zero at its first k-step
          if constexpr (FMT == TDGEMM_I8)
            acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[ks][x], fb[yy], ks == 0 ? zero : acc[x][y],
                                                              0, 0, 0);
          else
            acc[x][y] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa[ks][x], fb[yy], zero, 0, 0, 0,
                                                                          127, 0, 127);
        }
    }
  };
  // C = fma(r, inv, C) for the half h of the pair just multiplied (eqs. 5, 2)
  auto epi_half = [&](float inv, auto hc) {
    constexpr int h = decltype(hc)::value;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          cacc[x][2 * h + yy][r] = __builtin_fmaf((float)acc[x][2 * h + yy][r], inv, cacc[x][2 * h + yy][r]);
  };
  const std::integral_constant<int, 0> H0;
  const std::integral_constant<int, 1> H1;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int64_t l = 0; l < a.nL; ++l) {
    const int buf = (int)(l & 1);
    const int64_t pair = (i * a.nJ + j) * a.nL + l;
    if (l + 1 < a.nL) gload(l + 1);
    read_a(buf);
    if constexpr (STAGED) {
      mma_half(buf, H0);
      mma_half(buf, H1);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wr * 64 + x * 16 + 4 * g + r, col = wc * 64 + y * 16 + li;
            const int64_t o = pair * (kL8 * kL8) + row * kL8 + col;
            if constexpr (FMT == TDGEMM_I8) static_cast<int32_t *>(a.out)[o] = acc[x][y][r];
            else                            static_cast<float *>(a.out)[o] = acc[x][y][r];
          }
    } else {
      const float inv = (float)a.pairs[pair].inv;
      mma_half(buf, H0);
      mma_half(buf, H1);
      epi_half(inv, H0);
      epi_half(inv, H1);
    }
    if (l + 1 < a.nL) sstore(buf ^ 1);
    lds_barrier();
  }
  if constexpr (!STAGED) {
    float *C = static_cast<float *>(a.out);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = i * kL8 + wr * 64 + x * 16 + 4 * g + r;
          const int64_t n = j * kL8 + wc * 64 + y * 16 + li;
          if (m < a.M && n < a.N) C[m * a.ldc + n] = cacc[x][y][r];
        }
  }
}

// C = fma(float(R_pair), float(inv_pair), C), l ascending from 0, from staged products.
template <int FMT>
__global__ __launch_bounds__(kThreads) void k_scale_sum8(Gemm8Args a) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= a.M * a.N) return;
  const int64_t m = e / a.N, n = e - (e / a.N) * a.N;
  const int64_t i = m / kL8, j = n / kL8;
  const int r = (int)(m - i * kL8), c = (int)(n - j * kL8);
  float acc = 0.f;
  for (int64_t l = 0; l < a.nL; ++l) {
    const int64_t pair = (i * a.nJ + j) * a.nL + l;
    const int64_t o = pair * (kL8 * kL8) + r * kL8 + c;
    const float rv = (FMT == TDGEMM_I8) ? (float)static_cast<const int32_t *>(a.in)[o]
                                        : static_cast<const float *>(a.in)[o];
    acc = __builtin_fmaf(rv, (float)a.pairs[pair].inv, acc);
  }
  static_cast<float *>(a.out)[m * a.ldc + n] = acc;
}

// ---------------------------------------------------------------------------
hipError_t launch_quant8(const Quant8Args &a, int in_dtype, int fmt, hipStream_t st) {
  const int64_t blocks = a.nI * a.nL + a.nL * a.nJ;
  if (blocks == 0) return hipSuccess;
  const dim3 grid((unsigned)blocks), blk(kThreads);
  if (in_dtype == TDGEMM_F64) {
    if (fmt == TDGEMM_I8) hipLaunchKernelGGL((k_quant8<double, TDGEMM_I8>), grid, blk, 0, st, a);
    else                  hipLaunchKernelGGL((k_quant8<double, TDGEMM_E4M3>), grid, blk, 0, st, a);
  } else {
    if (fmt == TDGEMM_I8) hipLaunchKernelGGL((k_quant8<float, TDGEMM_I8>), grid, blk, 0, st, a);
    else                  hipLaunchKernelGGL((k_quant8<float, TDGEMM_E4M3>), grid, blk, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_gemm8(const Gemm8Args &a, int fmt, bool staged, hipStream_t st) {
  const int64_t tiles = a.nI * a.nJ;
  if (tiles == 0 || a.nL == 0) return hipSuccess;
  const dim3 grid((unsigned)((tiles + 7) / 8 * 8)), blk(kThreads);   // whole XCD ranges
  if (fmt == TDGEMM_I8) {
    if (staged) hipLaunchKernelGGL((k_gemm8<TDGEMM_I8, true>), grid, blk, 0, st, a);
    else        hipLaunchKernelGGL((k_gemm8<TDGEMM_I8, false>), grid, blk, 0, st, a);
  } else {
    if (staged) hipLaunchKernelGGL((k_gemm8<TDGEMM_E4M3, true>), grid, blk, 0, st, a);
    else        hipLaunchKernelGGL((k_gemm8<TDGEMM_E4M3, false>), grid, blk, 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_scale_sum8(const Gemm8Args &a, int fmt, hipStream_t st) {
  const int64_t n = a.M * a.N;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), blk(kThreads);
  if (fmt == TDGEMM_I8) hipLaunchKernelGGL((k_scale_sum8<TDGEMM_I8>), grid, blk, 0, st, a);
  else                  hipLaunchKernelGGL((k_scale_sum8<TDGEMM_E4M3>), grid, blk, 0, st, a);
  return hipGetLastError();
}

}  // namespace tdg
