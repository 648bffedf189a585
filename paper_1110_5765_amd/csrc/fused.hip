// Fused throughput-distortion GEMM: every stage of a subblock pair in one
// kernel (Sec. 3 with the settings of Sec. 5.B / Sec. 6).
//
// One workgroup (L / 16 wavefronts) computes one L x L inner kernel R_ij and walks
// its pairs l = 0, 1, ... in order. Each pair's K extent is cut into chunks of
// 16 raw columns. For every chunk the threads load raw A / B values from HBM,
// compand them (eq. 3) and pack them (eqs. 6-7, or 11) straight into a
// double-buffered LDS tile; wave w then runs FP64 (or FP32) 16x16x4 MFMAs for
// output columns 16w..16w+15, accumulating the packed product over the
// packed index in ascending order. After a pair's last chunk the packed result
// is unpacked in registers (eqs. 9-10 or 13-14), reverse-companded (eq. 5) and
// added to a register-resident C tile (eq. 2). W = 1 pairs run the plain
// product. C is written once at the end.
//
// Row placement: lane (g = lane / 16, c = lane % 16) keeps, for row block rb
// and register r, the C element of tile row 16 rb + 4 g + r. The LDS row of the
// A operand that feeds that result slot is permuted accordingly, which for the
// asymmetric form also routes the W rows unpacked from one packed word to the
// same lane whatever the pair's W.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace tdg {

// position (0..15) of the A-operand row that produces lane group g, register r
template <typename PT> __device__ __forceinline__ int mfma_pos(int g, int r);
template <> __device__ __forceinline__ int mfma_pos<double>(int g, int r) { return g + 4 * r; }
template <> __device__ __forceinline__ int mfma_pos<float>(int g, int r) { return 4 * g + r; }

// (g, r) owning packed row ml (0..15 within its 16-row block) of packing W:
// its unpacked rows W*ml + s are the rows 4g + r' of the C slots.
__device__ __forceinline__ void owner_of_packed_row(int ml, int W, int &g, int &r) {
  if (W == 1)      { g = ml >> 2;        r = ml & 3; }
  else if (W == 2) { g = (ml & 7) >> 1;  r = ((ml >> 3) << 1) | (ml & 1); }
  else             { g = ml & 3;         r = ml >> 2; }
}

template <typename PT>
__device__ __forceinline__ int lds_row_of(int m, int W) {
  int g, r;
  owner_of_packed_row(m & 15, W, g, r);
  return (m & ~15) + mfma_pos<PT>(g, r);
}

template <typename PT>
__device__ __forceinline__ PT compand_v(PT x, PT c, int W) {
  return (W == 1) ? x : rint(c * x);
}

template <typename IT, typename PT, int L, int FORM, bool TA, bool TB>
__global__ __launch_bounds__(4 * L) void k_fused(GemmOperands g, const IT *__restrict__ A,
                                                    const IT *__restrict__ B, PT *__restrict__ C,
                                                    int64_t ntiles, int64_t per_xcd) {
  constexpr int NT = 4 * L;           // threads: L / 16 wavefronts, one 16-column strip each
  constexpr int RB = L / 16;          // 16-row blocks of the tile
  constexpr int CB = 1;               // 16-column blocks per wave
  constexpr int V = 16 * L / NT;      // raw values per thread per operand per chunk (4)
  constexpr int SA = 17;              // LDS row stride of the A chunk (odd: no bank conflicts)
  constexpr int SB = L + 1;
  constexpr int NCH = L / 16;         // chunks per pair
  typedef typename Mfma<PT>::Acc Acc;
  __shared__ PT sA[2][L * SA];
  __shared__ PT sB[2][16 * SB];

  // XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so
  // give each XCD a contiguous range, grouped 8 tile-rows at a time (shared
  // B panels, then A panels, stay in that XCD's L2).
  const int64_t bid = blockIdx.x;
  const int64_t lin = (bid & 7) * per_xcd + (bid >> 3);
  if (lin >= ntiles) return;
  const Problem &pb = g.pb;
  constexpr int64_t GROUP = 8;
  const int64_t grp = lin / (GROUP * pb.nJ);
  const int64_t first_i = grp * GROUP;
  const int64_t gsize = min(GROUP, pb.nI - first_i);
  const int64_t in_grp = lin - grp * GROUP * pb.nJ;
  const int64_t ti = first_i + in_grp % gsize;
  const int64_t tj = in_grp / gsize;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lg = lane >> 4, lc = lane & 15;
  const int wcol = wave * 16;
  const int64_t r0 = ti * L, c0 = tj * L;
  const tdgemm_pair *prs = g.pairs + (ti * pb.nJ + tj) * pb.nL;

  Acc accR[RB][CB], accC[RB][CB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) { accR[a][b] = Mfma<PT>::zero(); accC[a][b] = Mfma<PT>::zero(); }

  PT ra[V], rb[V];

  // --- raw loads of chunk (l, kc) ---------------------------------------
  auto load_chunk = [&](int64_t l, int kc, int W) {
    const int64_t k0 = l * L + kc * 16;
    const bool colseg = (FORM == TDGEMM_ASYM) && W > 1;
    if (!colseg) {                        // thread: one row m, V consecutive k
      if (!TA) {
        const int m = tid / (16 / V), ks0 = (tid % (16 / V)) * V;
        const int64_t row = r0 + m;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const int64_t col = k0 + ks0 + q;
          ra[q] = (row < pb.M && col < pb.K) ? (PT)A[row * pb.lda + col] : (PT)0;
        }
      } else {
        const int m = tid % L, ks0 = (tid / L) * V;
        const int64_t row = r0 + m;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const int64_t col = k0 + ks0 + q;
          ra[q] = (row < pb.M && col < pb.K) ? (PT)A[col * pb.lda + row] : (PT)0;
        }
      }
    } else {                              // thread: one column k, V consecutive rows
      if (!TA) {
        const int k = tid % 16, ms0 = (tid / 16) * V;
        const int64_t col = k0 + k;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const int64_t row = r0 + ms0 + q;
          ra[q] = (row < pb.M && col < pb.K) ? (PT)A[row * pb.lda + col] : (PT)0;
        }
      } else {
        const int k = tid / (NT / 16), ms0 = (tid % (NT / 16)) * V;
        const int64_t col = k0 + k;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const int64_t row = r0 + ms0 + q;
          ra[q] = (row < pb.M && col < pb.K) ? (PT)A[col * pb.lda + row] : (PT)0;
        }
      }
    }
    if (!TB) {                            // thread: one column n, V consecutive k
      const int n = tid % L, ks0 = (tid / L) * V;
      const int64_t col = c0 + n;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int64_t row = k0 + ks0 + q;
        rb[q] = (row < pb.K && col < pb.N) ? (PT)B[row * pb.ldb + col] : (PT)0;
      }
    } else {
      const int n = tid / (16 / V), ks0 = (tid % (16 / V)) * V;
      const int64_t col = c0 + n;
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int64_t row = k0 + ks0 + q;
        rb[q] = (row < pb.K && col < pb.N) ? (PT)B[col * pb.ldb + row] : (PT)0;
      }
    }
  };

  // --- compand + pack the registers into LDS buffer `buf` -----------------
  // W is a template constant here so that the register arrays are indexed
  // with constants only.
  auto store_chunk_w = [&](auto wc, int buf, PT ca, PT cbv, PT z, PT zi) {
    constexpr int W = decltype(wc)::value;
    constexpr bool colseg = (FORM == TDGEMM_ASYM) && W > 1;
    PT *a_s = sA[buf];
    PT *b_s = sB[buf];
    if (!colseg) {
      int m, ks0;
      if (!TA) { m = tid / (16 / V); ks0 = (tid % (16 / V)) * V; }
      else     { m = tid % L;        ks0 = (tid / L) * V; }
      const int row = lds_row_of<PT>(m, 1);
      if (W == 1) {
#pragma unroll
        for (int q = 0; q < V; ++q) a_s[row * SA + ks0 + q] = ra[q];
      } else {                            // eq. (6): W consecutive columns per word
#pragma unroll
        for (int u = 0; u < V / W; ++u) {
          PT acc = compand_v(ra[u * W + W - 1], ca, W);
#pragma unroll
          for (int s = W - 2; s >= 0; --s) acc = acc * z + compand_v(ra[u * W + s], ca, W);
          a_s[row * SA + ks0 / W + u] = acc;
        }
      }
    } else {                              // eq. (11): W consecutive rows per word
      int k, ms0;
      if (!TA) { k = tid % 16; ms0 = (tid / 16) * V; }
      else     { k = tid / (NT / 16); ms0 = (tid % (NT / 16)) * V; }
#pragma unroll
      for (int u = 0; u < V / W; ++u) {
        PT acc = compand_v(ra[u * W + W - 1], ca, W);
#pragma unroll
        for (int s = W - 2; s >= 0; --s) acc = acc * z + compand_v(ra[u * W + s], ca, W);
        a_s[lds_row_of<PT>(ms0 / W + u, W) * SA + k] = acc;
      }
    }
    int n, ks0;
    if (!TB) { n = tid % L;        ks0 = (tid / L) * V; }
    else     { n = tid / (16 / V); ks0 = (tid % (16 / V)) * V; }
    if (FORM == TDGEMM_SYM && W > 1) {    // eq. (7): W consecutive rows per word, weights z^-i
#pragma unroll
      for (int u = 0; u < V / W; ++u) {
        PT acc = compand_v(rb[u * W + W - 1], cbv, W);
#pragma unroll
        for (int s = W - 2; s >= 0; --s) acc = acc * zi + compand_v(rb[u * W + s], cbv, W);
        b_s[(ks0 / W + u) * SB + n] = acc;
      }
    } else {
#pragma unroll
      for (int q = 0; q < V; ++q) b_s[(ks0 + q) * SB + n] = compand_v(rb[q], cbv, W);
    }
  };
  auto store_chunk = [&](int buf, int W, PT ca, PT cbv, PT z, PT zi) {
    if (W == 1) store_chunk_w(std::integral_constant<int, 1>(), buf, ca, cbv, z, zi);
    else if (W == 2) store_chunk_w(std::integral_constant<int, 2>(), buf, ca, cbv, z, zi);
    else store_chunk_w(std::integral_constant<int, 4>(), buf, ca, cbv, z, zi);
  };

  // --- MFMA over one chunk -------------------------------------------------
  auto mfma_chunk = [&](int buf, int W) {
    const PT *a_s = sA[buf];
    const PT *b_s = sB[buf];
    const bool sym = (FORM == TDGEMM_SYM) || W == 1;
    const int nks = sym ? 4 / W : 4;      // k-steps of 4 in this chunk
    const int rbn = sym ? RB : RB / W;    // output row blocks
    for (int ks = 0; ks < nks; ++ks) {
      PT af[RB], bf[CB];
#pragma unroll
      for (int a = 0; a < RB; ++a)
        if (a < rbn) af[a] = a_s[(16 * a + lc) * SA + 4 * ks + lg];
#pragma unroll
      for (int b = 0; b < CB; ++b) bf[b] = b_s[(4 * ks + lg) * SB + wcol + 16 * b + lc];
#pragma unroll
      for (int a = 0; a < RB; ++a)
        if (a < rbn)
#pragma unroll
          for (int b = 0; b < CB; ++b) accR[a][b] = Mfma<PT>::mma(af[a], bf[b], accR[a][b]);
    }
  };

  // --- unpack + reverse companding + l-sum ---------------------------------
  auto finish_pair = [&](int W, PT inv, PT z, PT zi) {
    if (W == 1) {
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) accC[a][b][r] = accC[a][b][r] + accR[a][b][r];
    } else if (FORM == TDGEMM_SYM) {      // eqs. (9)-(10), then eq. (5)
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT u = rint(accR[a][b][r]);
            const PT t = rint(z * u);
            const PT rr = u - zi * t;
            accC[a][b][r] = accC[a][b][r] + rr * inv;
          }
    } else if (W == 2) {                  // eqs. (13)-(14), two rows per word
#pragma unroll
      for (int a = 0; a < RB / 2; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT v = accR[a][b][r];
            const PT q0 = rint(v);
            const PT q1 = rint(zi * (v - q0));
            const int ra_ = 2 * a + (r >> 1), rr_ = (r & 1) * 2;
            accC[ra_][b][rr_] = accC[ra_][b][rr_] + q0 * inv;
            accC[ra_][b][rr_ + 1] = accC[ra_][b][rr_ + 1] + q1 * inv;
          }
    } else {                              // W == 4: four rows per word
#pragma unroll
      for (int a = 0; a < RB / 4; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT v = accR[a][b][r];
            const PT q0 = rint(v);
            const PT t1 = zi * (v - q0);
            const PT q1 = rint(t1);
            const PT t2 = zi * (t1 - q1);
            const PT q2 = rint(t2);
            const PT q3 = rint(zi * (t2 - q2));
            const int ra_ = 4 * a + r;
            accC[ra_][b][0] = accC[ra_][b][0] + q0 * inv;
            accC[ra_][b][1] = accC[ra_][b][1] + q1 * inv;
            accC[ra_][b][2] = accC[ra_][b][2] + q2 * inv;
            accC[ra_][b][3] = accC[ra_][b][3] + q3 * inv;
          }
    }
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) accR[a][b] = Mfma<PT>::zero();
  };

  // --- software pipeline over (l, chunk) ------------------------------------
  // The current pair's settings live in scalars: W, c_A, c_B, z, z^-1, inverse.
  int64_t l = 0;
  int kc = 0, buf = 0;
  int w = prs[0].w;
  PT ca = (PT)prs[0].c_a, cbv = (PT)prs[0].c_b, inv = (PT)prs[0].inv;
  PT z = (PT)ldexp(1.0, -prs[0].p), zi = (PT)ldexp(1.0, prs[0].p);
  load_chunk(0, 0, w);
  for (;;) {
    store_chunk(buf, w, ca, cbv, z, zi);
    __syncthreads();
    int64_t ln = l;
    int kcn = kc + 1;
    if (kcn == NCH) { ln = l + 1; kcn = 0; }
    const bool more = ln < pb.nL;
    int wn = w;
    if (more) {
      if (ln != l) wn = prs[ln].w;
      load_chunk(ln, kcn, wn);
    }
    mfma_chunk(buf, w);
    if (kc == NCH - 1) finish_pair(w, inv, z, zi);
    if (!more) break;
    if (ln != l) {
      w = wn;
      ca = (PT)prs[ln].c_a; cbv = (PT)prs[ln].c_b; inv = (PT)prs[ln].inv;
      z = (PT)ldexp(1.0, -prs[ln].p); zi = (PT)ldexp(1.0, prs[ln].p);
    }
    l = ln; kc = kcn; buf ^= 1;
  }

#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 16 * a + 4 * lg + r;
        const int64_t col = c0 + wcol + 16 * b + lc;
        if (row < pb.M && col < pb.N) C[row * pb.ldc + col] = accC[a][b][r];
      }
}

// ---------------------------------------------------------------------------
template <typename IT, typename PT, int L, int FORM>
static hipError_t launch_fused_t(const GemmOperands &g, const void *A, const void *B, void *C,
                                 hipStream_t st) {
  const int64_t ntiles = g.pb.nI * g.pb.nJ;
  const int64_t per_xcd = (ntiles + 7) / 8;
  const dim3 grid((unsigned)(per_xcd * 8));
  const dim3 block(4 * L);
  const IT *a = (const IT *)A;
  const IT *b = (const IT *)B;
  PT *c = (PT *)C;
  if (!g.ta && !g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, false, false>), grid, block, 0, st, g, a, b, c, ntiles, per_xcd);
  else if (g.ta && !g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, true, false>), grid, block, 0, st, g, a, b, c, ntiles, per_xcd);
  else if (!g.ta && g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, false, true>), grid, block, 0, st, g, a, b, c, ntiles, per_xcd);
  else
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, true, true>), grid, block, 0, st, g, a, b, c, ntiles, per_xcd);
  return hipGetLastError();
}

template <typename IT, typename PT>
static hipError_t launch_fused_l(const GemmOperands &g, const void *A, const void *B, void *C,
                                 hipStream_t st) {
  if (g.pb.L == 64)
    return g.form == TDGEMM_SYM ? launch_fused_t<IT, PT, 64, TDGEMM_SYM>(g, A, B, C, st)
                                : launch_fused_t<IT, PT, 64, TDGEMM_ASYM>(g, A, B, C, st);
  return g.form == TDGEMM_SYM ? launch_fused_t<IT, PT, 128, TDGEMM_SYM>(g, A, B, C, st)
                              : launch_fused_t<IT, PT, 128, TDGEMM_ASYM>(g, A, B, C, st);
}

hipError_t launch_fused(const GemmOperands &g, const void *A, const void *B, void *C, hipStream_t st) {
  if (g.in_dtype == TDGEMM_F64 && g.prec == TDGEMM_F64) return launch_fused_l<double, double>(g, A, B, C, st);
  if (g.in_dtype == TDGEMM_F32 && g.prec == TDGEMM_F64) return launch_fused_l<float, double>(g, A, B, C, st);
  return launch_fused_l<float, float>(g, A, B, C, st);
}

}  // namespace tdg
