// Fused throughput-distortion GEMM: every stage of a subblock pair in one
// kernel (Sec. 3 with the settings of Sec. 5.B / Sec. 6).
//
// A workgroup computes one inner kernel R_ij (an L x L tile of C) and walks
// its pairs l in ascending order -- all of them, or one group of consecutive l
// when the l-sum is split (the group sums are then added in order by
// k_sum_groups). Each pair's K extent is cut into chunks of KC raw columns (16
// or 48). For every chunk the threads load raw A / B values from HBM one or two
// chunks ahead, compand them (eq. 3) and pack them (eqs. 6-7, or 11) into a
// double-buffered LDS tile; each wavefront then runs FP64 (or FP32) 16x16x4
// MFMAs for its 16 RB x 16 CB part of the tile, accumulating the packed product
// over the packed index in ascending order. After a pair's last chunk the
// packed result is unpacked in registers (eqs. 9-10 or 13-14),
// reverse-companded (eq. 5) and added to a register-resident C tile (eq. 2) as
// C = fma(r, inv, C), one rounding per pair. W = 1 pairs run the plain
// product. C (or the group's partial result) is written once at the end.
//
// Row placement: lane (g = lane / 16, c = lane % 16) keeps, for its row block
// a and register r, the C element of tile row 16 a + 4 g + r of its wavefront
// (L = 64, 128) or 24 g + 4 a + r (L = 96). The LDS row of the A operand that
// feeds that result slot is permuted accordingly, which for the asymmetric
// form also routes the W rows unpacked from one packed word to the same lane
// whatever the pair's W.
//
// Thread layout of the raw loads (VA / VB values per thread and operand per
// chunk), independent of W so that prefetching may cross pairs:
//   A, symmetric form:  one row, consecutive columns (packs along columns);
//   A, asymmetric form: one column, consecutive rows (packs along rows);
//   B:                  one column, consecutive rows.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace tdg {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>());
    static_for<I + 1, N>(f);
  }
}

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

// L = 96: a wavefront owns 48 tile rows (three row blocks); its lane group g
// owns the 12 consecutive rows 12 g .. 12 g + 11 (slot (a, g, r) holds row
// 12 g + 4 a + r), so the W consecutive rows of an asymmetric word (W in
// {1, 2, 3, 4}, which all divide 12) stay in one lane. Packed row mb (W = 1:
// tile row) belongs to wavefront row mb / (48 / W); within it, to lane group g
// and word k = mb mod (12 / W), and goes to the MFMA position that yields that
// word's first slot. The packed rows of wavefront row wr start at LDS row
// 16 ceil(3 / W) wr (W = 1: 48 wr), where its MFMAs read them.
template <typename PT, int W>
__device__ __forceinline__ int lds_row_of96(int mb) {
  constexpr int per = 12 / W, rows = 48 / W, rbn = (3 + W - 1) / W;
  const int wr = mb / rows, mw = mb - wr * rows;
  const int g = mw / per, k = mw - g * per;
  return 16 * rbn * wr + 16 * (k >> 2) + mfma_pos<PT>(g, k & 3);
}

template <typename PT>
__device__ __forceinline__ int lds_row_of(int m, int W) {
  int g, r;
  owner_of_packed_row(m & 15, W, g, r);
  return (m & ~15) + mfma_pos<PT>(g, r);
}

// threads of a workgroup: L / 16 wavefronts; at L = 96 twelve wavefronts of
// 48 x 16, three on every SIMD
template <int L>
constexpr int fused_threads() { return L == 96 ? 768 : 4 * L; }

template <typename IT, typename PT, int L, int FORM, bool TA, bool TB>
struct Fused {
  static constexpr bool L96 = L == 96;
  // L = 128: one workgroup per inner kernel (128 x 128), so each subblock of A
  // and B is companded and packed once per inner kernel
  static constexpr bool WIDE = L == 128;
  static constexpr int TN = L96 ? 96 : (WIDE ? 128 : 64);  // output columns per workgroup
  static constexpr int NT = fused_threads<L>();
  static constexpr int WC = L96 ? 6 : 4;  // wavefront columns, 16 CB output columns each
  static constexpr int RB = L96 ? 3 : 4;  // 16-row blocks per wavefront
  static constexpr int CB = WIDE ? 2 : 1; // 16-column blocks per wavefront
  // raw inner columns per chunk: at L = 96, 48 (whole MFMA k-steps for every W
  // in {1, 2, 3, 4})
  static constexpr int KC = (L == 64 || WIDE) ? 16 : (L96 ? 48 : 32);
  // L = 96: the first half of the threads load A, the second half B, so that a
  // thread holds 12 values of one operand, whole packed words for every W
  static constexpr bool SPLIT = L96;
  static constexpr int NLD = SPLIT ? NT / 2 : NT;  // threads loading each operand
  static constexpr int VA = KC * L / NLD;  // raw A values per loading thread per chunk
  static constexpr int VB = KC * TN / NLD; // raw B values per loading thread per chunk
  static constexpr int WMAX = 4;           // packings {1, 2, 4}, and 3 at L = 96
  static constexpr bool HAS3 = L96;
  // packed accumulator sets: two let a pair's unpack overlap the next pair's
  // MFMAs (L = 64); with one (L = 96 and 128) a pair is unpacked right after
  // its own MFMAs
  static constexpr int NACC = (L96 || WIDE) ? 1 : 2;
  // LDS row strides in elements. A 64-bit fragment read serves 32 lanes at a
  // time over 64 four-byte banks: lane groups g = 0, 1 read rows lc = 0..15 at
  // column g (A) or column lc of rows g (B). With SA = KC + 2 (2 mod 32) the 32
  // A reads start on distinct even banks; with SB = TN + 16 (16 mod 32) the two
  // B rows fall on opposite halves of the banks.
  // L = 96: B rows are TN elements without padding (the two tiles would exceed
  // the 160 KB of LDS); element (k, n) sits at column n ^ 16 (k & 1) instead,
  // which puts the two B rows of a fragment read on opposite halves of the
  // banks.
  static constexpr int SA = KC + 2;
  static constexpr int SB = L96 ? TN : TN + 16;
  static constexpr int bcol(int k, int n) { return L96 ? (n ^ ((k & 1) << 4)) : n; }
  static constexpr int NCH = L / KC;      // chunks per pair
  // Symmetric form, A stored as given: four consecutive threads share a row and
  // thread i of the four holds columns 4i..4i+3 (and 4i+16..4i+19 when a chunk
  // has 32 columns), so each 16-byte load of a wavefront covers 64 contiguous
  // bytes of 16 rows and every packed word (W <= 4) lies in one thread.
  // (L = 96: thread i of the four holds columns 6i..6i+5.)
  static constexpr bool A_QUAD = FORM == TDGEMM_SYM && !TA;
  static constexpr bool A_SPLIT = A_QUAD && VA == 8;
  static constexpr int koffA(int v) { return A_SPLIT ? (v % 4) + 16 * (v / 4) : v; }
  // register sets of raw loads: the prefetch distance in chunks (one at L = 128,
  // where the 128 x 128 tile leaves fewer registers, and at L = 96, whose
  // 48-column chunks hold a whole chunk of matrix work)
  static constexpr int PF = (L96 || WIDE) ? 1 : 2;
  typedef typename Mfma<PT>::Acc Acc;
  static_assert(VA * NLD == KC * L && VB * NLD == KC * TN, "loads must cover a chunk");
  static_assert(KC % (4 * WMAX) == 0 && KC % 8 == 0 && (!HAS3 || KC % 12 == 0),
                "packed chunk depth: whole k-steps");
  static_assert(VA % WMAX == 0 && VA % 2 == 0 && VB % WMAX == 0 && VB % 2 == 0 &&
                (!HAS3 || (VA % 3 == 0 && VB % 3 == 0)),
                "a thread's raw values form whole packed words");
  static_assert(L96 ? (RB == 3) : (RB % WMAX == 0 && RB % 2 == 0),
                "asymmetric words: whole row blocks (L = 96: 12 rows per lane group)");
  static_assert(NT == 64 * WC * (L / (16 * RB)), "wavefront grid covers the tile");

  struct Smem {
    PT a[2][L * SA];
    PT b[2][KC * SB];
  };

  const Problem &pb;
  const IT *__restrict__ A;
  const IT *__restrict__ B;
  Smem &sm;
  int tid, lg, lc, wr, wrow, wcol;
  int64_t r0, c0;
  int64_t kb = 0;         // inner index of the first subblock this workgroup sums
  // per-thread load coordinates inside a chunk
  int a_m, a_k;           // first (row, col) this thread loads from A's chunk
  int b_n, b_k;           // (col, first row) of B's chunk
  int offA, offB;         // byte offsets of (a_m, a_k) and (b_k, b_n) from the chunk corner
  bool a_row_ok, b_col_ok;
  bool lda_thread;        // loads (and packs) A; with SPLIT the others load B
  // SPLIT: W-independent parts of this thread's LDS word addresses, from which
  // each W forms its own with a few integer operations (see a_word, b_word)
  int q0, q1, q2;
  Acc accR[NACC][RB][CB], accC[RB][CB];   // accR[P]: packed product of the pairs of parity P
  // raw values of the next chunks; with SPLIT a thread holds one operand's, in ra
  PT ra[PF][VA], rb[SPLIT ? 1 : PF][SPLIT ? 1 : VB];
  __device__ __forceinline__ PT &raw_b(int s, int q) {
    if constexpr (SPLIT) return ra[s][q];
    else return rb[s][q];
  }

  __device__ __forceinline__ Fused(const Problem &pb_, const IT *A_, const IT *B_, Smem &sm_,
                                   int64_t r0_, int64_t c0_)
      : pb(pb_), A(A_), B(B_), sm(sm_), r0(r0_), c0(c0_) {
    tid = threadIdx.x;
    const int lane = tid & 63;
    lg = lane >> 4;
    lc = lane & 15;
    wr = (tid >> 6) / WC;
    wrow = wr * 16 * RB;
    wcol = ((tid >> 6) % WC) * 16 * CB;
    lda_thread = !SPLIT || tid < NLD;
    const int ta = tid;                               // index among the A loaders
    const int tb = SPLIT ? tid - NLD : tid;           // index among the B loaders
    if (FORM == TDGEMM_SYM) {
      // A as stored: four consecutive lanes share a row (16-byte loads of
      // consecutive columns, see A_QUAD); A transposed: consecutive lanes take
      // consecutive rows, which are consecutive in memory
      if (!TA) { a_m = ta >> 2;                         a_k = (ta & 3) * (A_SPLIT ? 4 : VA); }
      else     { a_m = ta % L;                      a_k = (ta / L) * VA; }
    } else {
      if (!TA) { a_k = ta % KC;        a_m = (ta / KC) * VA; }
      else     { a_k = ta / (L / VA);  a_m = (ta % (L / VA)) * VA; }
    }
    if (!TB) { b_n = tb % TN;         b_k = (tb / TN) * VB; }
    else     { b_n = tb / (KC / VB);  b_k = (tb % (KC / VB)) * VB; }
    offA = (TA ? a_k * (int)pb.lda + a_m : a_m * (int)pb.lda + a_k) * (int)sizeof(IT);
    offB = (TB ? b_n * (int)pb.ldb + b_k : b_k * (int)pb.ldb + b_n) * (int)sizeof(IT);
    a_row_ok = r0 + a_m < pb.M;
    b_col_ok = c0 + b_n < pb.N;
    if constexpr (SPLIT) {
      // a_k is a multiple of 12 and so are a_m (asymmetric) and b_k: the 12 / W
      // words of a thread are consecutive words of one row run (symmetric A),
      // of one lane group (asymmetric A) or of one column (B)
      if (lda_thread) {
        if (FORM == TDGEMM_SYM) { q0 = a_row<1>(a_m) * SA; q1 = a_k / 12; q2 = 0; }
        else { q0 = a_m / 48; q1 = mfma_pos<PT>((a_m % 48) / 12, 0); q2 = a_k; }
      } else {
        q0 = b_k / 12; q1 = b_n; q2 = 0;
      }
    }
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        accR[0][a][b] = Mfma<PT>::zero(); accR[NACC - 1][a][b] = Mfma<PT>::zero(); accC[a][b] = Mfma<PT>::zero();
      }
  }

  // One raw value: a buffer load from the chunk corner's resource, at this
  // thread's byte offset plus the value's uniform (scalar) byte offset, so no
  // load needs a per-lane 64-bit address.
  __device__ __forceinline__ static PT raw_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (sizeof(IT) == 8)
      return (PT)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
      return (PT)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }

  // Raw loads of the chunk starting at inner index k0: the chunk corner as a
  // buffer resource spanning L rows (or columns) of the operand, plus this
  // thread's fixed offset (L ld sizeof(IT) < 2^30, checked on the host). With
  // CHECK, out-of-range elements read 0 and are never loaded.
  template <bool CHECK, int S>
  __device__ __forceinline__ void load(int64_t kc0) {
    const int64_t k0 = kb + kc0;
    const IT *Ab = TA ? A + k0 * pb.lda + r0 : A + r0 * pb.lda + k0;
    const IT *Bb = TB ? B + c0 * pb.ldb + k0 : B + k0 * pb.ldb + c0;
    const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
        (void *)Ab, (short)0, (int)((int64_t)L * pb.lda * (int64_t)sizeof(IT)), kBufWord3);
    const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
        (void *)Bb, (short)0, (int)((int64_t)L * pb.ldb * (int64_t)sizeof(IT)), kBufWord3);
    const int64_t kleft = pb.K - k0, mleft = pb.M - r0;
    const int krem = CHECK ? (int)(kleft < KC ? kleft : KC) : KC;     // valid inner columns (may be <= 0)
    const int mrem = CHECK ? (int)(mleft < L ? mleft : L) : L;        // valid rows of the tile
    // value q of a thread sits at a uniform distance q * step from its first one:
    // a scalar base per q and one per-thread offset for all of them
    constexpr bool sym = FORM == TDGEMM_SYM;
    const int64_t stepA = sym ? (TA ? pb.lda : 1) : (TA ? 1 : pb.lda);
    const int64_t stepB = TB ? 1 : pb.ldb;
    // Where a thread's values are consecutive in memory (symmetric A as stored,
    // asymmetric A transposed, B transposed), G of them come in one 16-byte load
    // (runs of 4 for koffA).
    constexpr int G = 16 / (int)sizeof(IT);
    constexpr bool WIDE_A = (sym != TA) && VA % G == 0 && (!A_SPLIT || G <= 4);
    constexpr bool WIDE_B = TB && VB % G == 0;
    typedef IT vec_t __attribute__((ext_vector_type(G)));
    if (lda_thread) {
      if constexpr (WIDE_A && !CHECK) {
#pragma unroll
        for (int q = 0; q < VA; q += G) {
          const vec_t v = __builtin_bit_cast(
              vec_t, __builtin_amdgcn_raw_buffer_load_b128(rA, offA, koffA(q) * (int)sizeof(IT), 0));
#pragma unroll
          for (int e = 0; e < G; ++e) ra[S][q + e] = (PT)v[e];
        }
      } else {
#pragma unroll
        for (int q = 0; q < VA; ++q) {
          // symmetric: (row a_m, col a_k + q); asymmetric: (row a_m + q, col a_k)
          bool ok = true;
          if (CHECK) ok = sym ? (a_row_ok && a_k + koffA(q) < krem) : (a_m + q < mrem && a_k < krem);
          ra[S][q] = ok ? raw_load(rA, offA, (int)(koffA(q) * stepA * (int64_t)sizeof(IT))) : (PT)0;
        }
      }
    }
    if (!SPLIT || !lda_thread) {
      if constexpr (WIDE_B && !CHECK) {
#pragma unroll
        for (int q = 0; q < VB; q += G) {
          const vec_t v = __builtin_bit_cast(
              vec_t, __builtin_amdgcn_raw_buffer_load_b128(rB, offB, q * (int)sizeof(IT), 0));
#pragma unroll
          for (int e = 0; e < G; ++e) raw_b(S, q + e) = (PT)v[e];
        }
      } else {
#pragma unroll
        for (int q = 0; q < VB; ++q) {
          const bool ok = !CHECK || (b_col_ok && b_k + q < krem);
          raw_b(S, q) = ok ? raw_load(rB, offB, (int)(q * stepB * (int64_t)sizeof(IT))) : (PT)0;
        }
      }
    }
  }

  template <int W>
  __device__ __forceinline__ static PT compand(PT x, PT c) { return (W == 1) ? x : rint(c * x); }

  // Compand + pack register set S into LDS buffer `buf`, one packed word per
  // "unit": units 0..UA-1 are words of A (eq. 6 along columns, or eq. 11 along
  // rows), the rest words of B (eq. 7, or unpacked B). Packing words are
  // evaluated by Horner's rule from the highest slot; the products with z are
  // exact (powers of two), so each step is one fused multiply-add.
  template <int W>
  static constexpr int units_a() { return VA / W; }
  template <int W>
  static constexpr int units_b() { return (FORM == TDGEMM_SYM && W > 1) ? VB / W : VB; }

  // LDS row of packed A row mb (W = 1: tile row)
  template <int W>
  __device__ __forceinline__ static int a_row(int mb) {
    if constexpr (L96) return lds_row_of96<PT, W>(mb);
    else return lds_row_of<PT>(mb, W);
  }

  // LDS element index of word u of this thread (A: unit u, B: unit u past A's)
  template <int W, int u>
  __device__ __forceinline__ int a_word(void) const {
    if constexpr (SPLIT) {
      if constexpr (FORM == TDGEMM_SYM) return q0 + q1 * (12 / W) + u;
      constexpr int rbn = (RB + W - 1) / W;      // the same row as lds_row_of96<PT, W>
      return (16 * rbn * q0 + q1 + 16 * (u >> 2) + mfma_pos<PT>(0, u & 3)) * SA + q2;
    } else {
      if constexpr (FORM == TDGEMM_SYM) return a_row<1>(a_m) * SA + (a_k + koffA(u * W)) / W;
      else return a_row<W>(a_m / W + u) * SA + a_k;
    }
  }
  template <int W, int u>
  __device__ __forceinline__ int b_word(void) const {
    if constexpr (SPLIT) {
      const int k = ((FORM == TDGEMM_SYM && W > 1) ? q0 * (12 / W) : q0 * 12) + u;
      return k * SB + bcol(k, q1);
    } else {
      const int k = ((FORM == TDGEMM_SYM && W > 1) ? b_k / W : b_k) + u;
      return k * SB + bcol(k, b_n);
    }
  }

  template <int W, int S, int U>
  __device__ __forceinline__ void unit(int buf, PT ca, PT cb, PT z, PT zi) {
    if (U < units_a<W>()) {
      constexpr int u = U;
      PT acc = compand<W>(ra[S][u * W + W - 1], ca);
#pragma unroll
      for (int s = W - 2; s >= 0; --s) acc = __builtin_fma(acc, z, compand<W>(ra[S][u * W + s], ca));
      sm.a[buf][a_word<W, u>()] = acc;
    } else {
      constexpr int u = U - units_a<W>();
      if (FORM == TDGEMM_SYM && W > 1) {
        PT acc = compand<W>(raw_b(S, u * W + W - 1), cb);
#pragma unroll
        for (int s = W - 2; s >= 0; --s) acc = __builtin_fma(acc, zi, compand<W>(raw_b(S, u * W + s), cb));
        sm.b[buf][b_word<W, u>()] = acc;
      } else {
        sm.b[buf][b_word<W, u>()] = compand<W>(raw_b(S, u), cb);
      }
    }
  }

  template <int W, int S, int U0, int U1>
  __device__ __forceinline__ void units(int buf, PT ca, PT cb, PT z, PT zi) {
    if constexpr (U0 < U1) {
      unit<W, S, U0>(buf, ca, cb, z, zi);
      units<W, S, U0 + 1, U1>(buf, ca, cb, z, zi);
    }
  }

  template <int W, int S>
  __device__ __forceinline__ void store(int buf, PT ca, PT cb, PT z, PT zi) {
    if constexpr (SPLIT) {
      // Left loop-invariant, the word addresses of all four W would be hoisted
      // out of the pair loop and kept live together, past the 168 registers of
      // three wavefronts per SIMD; an empty asm statement makes their inputs
      // opaque here, so each W forms its own (a few integer operations) in place.
      asm volatile("" : "+v"(q0), "+v"(q1), "+v"(q2));
      if (lda_thread) units<W, S, 0, units_a<W>()>(buf, ca, cb, z, zi);
      else units<W, S, units_a<W>(), units_a<W>() + units_b<W>()>(buf, ca, cb, z, zi);
    } else {
      units<W, S, 0, units_a<W>() + units_b<W>()>(buf, ca, cb, z, zi);
    }
  }

  // The chunk's MFMAs into accumulator set P: packed depth KC / W (symmetric)
  // or KC (asymmetric, W = 1). Wavefront (wr, wc) multiplies packed row blocks
  // of its 64 output rows by its column blocks. B fragment rows are 4 ks + lg,
  // of the parity of lg.
  template <int W, int P>
  __device__ __forceinline__ void mma(int buf) {
    constexpr bool SYMW = (FORM == TDGEMM_SYM) || W == 1;
    constexpr int NKS = SYMW ? KC / (4 * W) : KC / 4;
    constexpr int RBN = SYMW ? RB : (RB + W - 1) / W;
    const PT *as = sm.a[buf] + (16 * RBN * wr + lc) * SA + lg;
    const PT *bs = sm.b[buf] + lg * SB + lc;
    // one fragment set: the reads of k-step ks + 1 go out right after the
    // MFMAs of ks are issued and return while those execute
    static_for<0, NKS>([&](auto ksc) {
      constexpr int ks = decltype(ksc)::value;
      PT af[RBN], bf[CB];
#pragma unroll
      for (int a = 0; a < RBN; ++a) af[a] = as[16 * a * SA + 4 * ks];
#pragma unroll
      for (int b = 0; b < CB; ++b) bf[b] = bs[4 * ks * SB + bcol(lg, wcol + 16 * b)];
#pragma unroll
      for (int a = 0; a < RBN; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
          accR[P][a][b] = Mfma<PT>::mma(af[a], bf[b], accR[P][a][b]);
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  // unpack + reverse companding + l-sum of the pair held in accumulator set P
  template <int W, int P>
  __device__ __forceinline__ void finish(PT inv, PT z, PT zi) {
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if (W == 1) {
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) accC[a][b][r] = accC[a][b][r] + accR[P][a][b][r];
      } else if (FORM == TDGEMM_SYM) {           // eqs. (9)-(10), then eq. (5)
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT u = rint(accR[P][a][b][r]);
            const PT t = rint(z * u);
            const PT rr = __builtin_fma(-zi, t, u);     // exact: zi * t is a power-of-two multiple
            accC[a][b][r] = __builtin_fma(rr, inv, accC[a][b][r]);
          }
      } else if (L96) {                          // eqs. (13)-(14): W rows per word
        // word k = 4 a + r of a lane group (k < 12 / W) yields its rows W k + s,
        // in the slots (W k + s) / 4, register (W k + s) mod 4
#pragma unroll
        for (int a = 0; a < (RB + W - 1) / W; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (4 * a + r >= 4 * RB / W) continue;
            PT t = accR[P][a][b][r];
#pragma unroll
            for (int sl = 0; sl < W; ++sl) {
              const PT q = rint(t);
              const int o = W * (4 * a + r) + sl;
              accC[o >> 2][b][o & 3] = __builtin_fma(q, inv, accC[o >> 2][b][o & 3]);
              if (sl + 1 < W) t = zi * (t - q);
            }
          }
      } else if (W == 2) {                       // eqs. (13)-(14), two rows per word
#pragma unroll
        for (int a = 0; a < RB / 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT v = accR[P][a][b][r];
            const PT q0 = rint(v);
            const PT q1 = rint(zi * (v - q0));
            const int ra_ = 2 * a + (r >> 1), rr_ = (r & 1) * 2;
            accC[ra_][b][rr_] = __builtin_fma(q0, inv, accC[ra_][b][rr_]);
            accC[ra_][b][rr_ + 1] = __builtin_fma(q1, inv, accC[ra_][b][rr_ + 1]);
          }
      } else {                                   // W == 4: four rows per word
#pragma unroll
        for (int a = 0; a < RB / 4; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const PT v = accR[P][a][b][r];
            const PT q0 = rint(v);
            const PT t1 = zi * (v - q0);
            const PT q1 = rint(t1);
            const PT t2 = zi * (t1 - q1);
            const PT q2 = rint(t2);
            const PT q3 = rint(zi * (t2 - q2));
            const int ra_ = 4 * a + r;
            accC[ra_][b][0] = __builtin_fma(q0, inv, accC[ra_][b][0]);
            accC[ra_][b][1] = __builtin_fma(q1, inv, accC[ra_][b][1]);
            accC[ra_][b][2] = __builtin_fma(q2, inv, accC[ra_][b][2]);
            accC[ra_][b][3] = __builtin_fma(q3, inv, accC[ra_][b][3]);
          }
      }
    }
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) accR[P][a][b] = Mfma<PT>::zero();
  }

  struct PairState {
    int w;
    PT ca, cb, z, zi, inv;
  };

  __device__ __forceinline__ static PairState pair_state(const tdgemm_pair &o) {
    PairState ps;
    ps.w = o.w;
    ps.ca = (PT)o.c_a; ps.cb = (PT)o.c_b; ps.inv = (PT)o.inv;
    // z = 2^-p and 1/z = 2^p built from exponent bits (integer work, so the
    // wavefront-uniform state can live in scalar registers); |p| < 1022
    ps.z = (PT)__builtin_bit_cast(double, (uint64_t)(1023 - o.p) << 52);
    ps.zi = (PT)__builtin_bit_cast(double, (uint64_t)(1023 + o.p) << 52);
    return ps;
  }

  template <int S>
  __device__ __forceinline__ void store_any(int buf, const PairState &ps) {
    if (ps.w == 2) store<2, S>(buf, ps.ca, ps.cb, ps.z, ps.zi);
    else if (ps.w == 1) store<1, S>(buf, ps.ca, ps.cb, ps.z, ps.zi);
    else if constexpr (HAS3 && WMAX == 4) {
      if (ps.w == 3) store<3, S>(buf, ps.ca, ps.cb, ps.z, ps.zi);
      else store<4, S>(buf, ps.ca, ps.cb, ps.z, ps.zi);
    } else store<WMAX, S>(buf, ps.ca, ps.cb, ps.z, ps.zi);
  }

  template <int P>
  __device__ __forceinline__ void mma_any(int buf, int w) {
    if (w == 2) mma<2, P>(buf);
    else if (w == 1) mma<1, P>(buf);
    else if constexpr (HAS3 && WMAX == 4) {
      if (w == 3) mma<3, P>(buf);
      else mma<4, P>(buf);
    } else mma<WMAX, P>(buf);
  }

  template <int P>
  __device__ __forceinline__ void finish_any(const PairState &ps) {
    if (ps.w == 2) finish<2, P>(ps.inv, ps.z, ps.zi);
    else if (ps.w == 1) finish<1, P>(ps.inv, ps.z, ps.zi);
    else if constexpr (HAS3 && WMAX == 4) {
      if (ps.w == 3) finish<3, P>(ps.inv, ps.z, ps.zi);
      else finish<4, P>(ps.inv, ps.z, ps.zi);
    } else finish<WMAX, P>(ps.inv, ps.z, ps.zi);
  }

  // Chunk g of the pair in accumulator set P (two sets): compand + pack
  // register set S into LDS buffer g % 2, barrier, issue the raw loads of chunk
  // g + PF into set S (PF chunks of matrix work before they are needed), run
  // chunk g's MFMAs. In the first chunk of a pair the previous pair, in set
  // 1 - P, is unpacked right after these MFMAs are issued (measured faster than
  // unpacking first).
  template <bool CHECK, int S, int P>
  __device__ __forceinline__ void iter(int64_t g, int64_t total, const PairState &ps,
                                       const PairState &prev, bool finish_prev) {
    const int buf = (int)(g & 1);
    store_any<S>(buf, ps);
    lds_barrier();
    // always issued (the last chunk again past the end), so that the number of
    // loads in flight is the same on every path and waits count exactly
    const int64_t g2 = g + PF < total ? g + PF : total - 1;
    load<CHECK, S>((g2 / NCH) * L + (g2 % NCH) * KC);
    mma_any<P>(buf, ps.w);
    if (finish_prev) finish_any<1 - P>(prev);
  }

  // All chunks of pair l (NCH is even, so chunk parity restarts with each pair).
  template <bool CHECK, int P>
  __device__ __forceinline__ void pair(int64_t l, int64_t total, PairState &ps, PairState &prev,
                                       const tdgemm_pair *prs) {
    prev = ps;
    ps = pair_state(prs[l]);
    const int64_t g0 = l * NCH;
    iter<CHECK, 0, P>(g0, total, ps, prev, l > 0);
    iter<CHECK, PF - 1, P>(g0 + 1, total, ps, prev, false);
#pragma unroll 1
    for (int kc = 2; kc < NCH; kc += 2) {
      iter<CHECK, 0, P>(g0 + kc, total, ps, prev, false);
      iter<CHECK, PF - 1, P>(g0 + kc + 1, total, ps, prev, false);
    }
  }

  // One accumulator set: pair l with its packing W fixed for all of its chunks,
  // unpacked right after its last MFMAs. Dispatching on W once per pair (not
  // per stage of a chunk) keeps the register allocation of each W separate;
  // per stage, the 128 x 128 tile spills.
  template <bool CHECK, int W>
  __device__ __forceinline__ void pair_w(int64_t l, int64_t total, const PairState &ps) {
    const int64_t g0 = l * NCH;
#pragma unroll 1
    for (int kc = 0; kc < NCH; kc += 2) {
      static_for<0, 2>([&](auto hc) {
        constexpr int h = decltype(hc)::value;   // LDS buffer of chunk g0 + kc + h
        constexpr int S = PF == 2 ? h : 0;        // register set of its raw values
        store<W, S>(h, ps.ca, ps.cb, ps.z, ps.zi);
        lds_barrier();
        const int64_t g = g0 + kc + h;
        const int64_t g2 = g + PF < total ? g + PF : total - 1;
        load<CHECK, S>((g2 / NCH) * L + (g2 % NCH) * KC);
        mma<W, 0>(h);
      });
    }
    finish<W, 0>(ps.inv, ps.z, ps.zi);
  }

  template <bool CHECK>
  __device__ __forceinline__ void pair1(int64_t l, int64_t total, const tdgemm_pair *prs) {
    const PairState ps = pair_state(prs[l]);
    if (ps.w == 2) pair_w<CHECK, 2>(l, total, ps);
    else if (ps.w == 1) pair_w<CHECK, 1>(l, total, ps);
    else if constexpr (HAS3 && WMAX == 4) {
      if (ps.w == 3) pair_w<CHECK, 3>(l, total, ps);
      else pair_w<CHECK, 4>(l, total, ps);
    } else pair_w<CHECK, WMAX>(l, total, ps);
  }

  // Walk all pairs of the tile. A tile inside M and N needs bounds checks only
  // for chunks that reach past K (chunk g starts at inner index g KC): pairs
  // whose prefetches all stay inside K run unchecked, the rest checked.
  template <bool CHECK>
  __device__ __forceinline__ void run(const tdgemm_pair *prs, int64_t nL) {
    if constexpr (NACC == 1) run1<CHECK>(prs, nL);
    else run2<CHECK>(prs, nL);
  }

  // One accumulator set: pair after pair.
  template <bool CHECK>
  __device__ __forceinline__ void run1(const tdgemm_pair *prs, int64_t nL) {
    const int64_t total = nL * NCH;
    const int64_t kfull = (pb.K - kb) / KC;                           // chunks inside K
    const int64_t tail = CHECK ? 0 : (kfull < total ? kfull : total);  // first chunk crossing K
    if (tail > 0) load<false, 0>(0); else load<true, 0>(0);
    if (PF == 2 && total > 1) { if (tail > 1) load<false, PF - 1>(KC); else load<true, PF - 1>(KC); }
    // pair l prefetches up to chunk (l + 1) NCH + PF - 1
    const int64_t l1 = tail >= PF ? (tail - PF) / NCH : 0;
    int64_t l = 0;
    for (; l < l1; ++l) pair1<false>(l, total, prs);
    for (; l < nL; ++l) pair1<true>(l, total, prs);
  }

  // Two accumulator sets: pairs in twos, each unpacked during the next one.
  template <bool CHECK>
  __device__ __forceinline__ void run2(const tdgemm_pair *prs, int64_t nL) {
    const int64_t total = nL * NCH;
    const int64_t kfull = (pb.K - kb) / KC;                           // chunks inside K
    const int64_t tail = CHECK ? 0 : (kfull < total ? kfull : total);  // first chunk crossing K
    if (tail > 0) load<false, 0>(0); else load<true, 0>(0);
    if (PF == 2 && total > 1) { if (tail > 1) load<false, PF - 1>(KC); else load<true, PF - 1>(KC); }
    // pair l prefetches up to chunk (l + 1) NCH + PF - 1
    int64_t l1 = tail >= PF ? (tail - PF) / NCH : 0;
    l1 -= l1 & 1;
    PairState ps = pair_state(prs[0]), prev = ps;
    int64_t l = 0;
    constexpr int P1 = NACC - 1;             // set of the odd pairs
    for (; l < l1; l += 2) {
      pair<false, 0>(l, total, ps, prev, prs);
      pair<false, P1>(l + 1, total, ps, prev, prs);
    }
    for (; l < nL; l += 2) {
      pair<true, 0>(l, total, ps, prev, prs);
      if (l + 1 < nL) pair<true, P1>(l + 1, total, ps, prev, prs);
    }
    if ((nL - 1) & 1) finish_any<P1>(ps);
    else finish_any<0>(ps);
  }

  __device__ __forceinline__ void write_c(PT *__restrict__ C, int64_t ldc) const {
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + wrow + (L96 ? 12 * lg + 4 * a : 16 * a + 4 * lg) + r;
          const int64_t col = c0 + wcol + 16 * b + lc;
          if (row < pb.M && col < pb.N) C[row * ldc + col] = accC[a][b][r];
        }
  }
};

template <typename IT, typename PT, int L, int FORM, bool TA, bool TB>
__global__ __launch_bounds__(fused_threads<L>(), (L == 64 ? 2 : 1)) void k_fused(GemmOperands g, const IT *__restrict__ A,
                                                 const IT *__restrict__ B, PT *__restrict__ C,
                                                 PT *__restrict__ part, int64_t ntiles,
                                                 int64_t ngroups, int64_t per_xcd) {
  typedef Fused<IT, PT, L, FORM, TA, TB> F;
  __shared__ typename F::Smem sm;
  // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so give
  // each XCD a contiguous range. Tiles go a few tile-rows at a time, so that the
  // workgroups running together on one XCD share A panels and B slabs in its L2.
  // A workgroup covers L rows and a TN-column slab of one inner kernel.
  const int64_t bid = blockIdx.x;
  const Problem &pb = g.pb;
  constexpr int64_t SLABS = L / F::TN;
  const int64_t nS = pb.nJ * SLABS;
  constexpr int64_t GROUP = (L == 64) ? 8 : 4;    // tile rows per group: an XCD's
  // tile t of a rows x cols grid in that order: concurrent workgroups form a GROUP x 8 block
  auto by_groups = [](int64_t t, int64_t rows, int64_t cols, int64_t &ti, int64_t &ts) {
    const int64_t grp = t / (GROUP * cols);
    const int64_t first_i = grp * GROUP;
    const int64_t gsize = min(GROUP, rows - first_i);
    const int64_t in_grp = t - grp * GROUP * cols;
    ti = first_i + in_grp % gsize;
    ts = in_grp / gsize;
  };
  int64_t grp_l = 0, ti, ts;
  // Each XCD runs per_xcd tiles, one per CU at a time (two at L = 64). When its last round
  // is full or at least half full, the border tiles (ragged M or N, less work)
  // of its share go last, in proportion to the share's size, so that the short
  // tiles end the launch. With only a few tiles in the last round, the row
  // order is kept: there the border tiles are better run beside the full tiles
  // of their own rows, whose operand panels the XCD's L2 still holds (measured
  // on 4000^3 and 3900^3 at L = 128 and on 4000^3, 4050^3, 4096^3 at L = 96).
  constexpr int64_t per_round = (L == 64) ? 64 : 32;   // workgroups an XCD runs at once
  const int64_t last = per_xcd % per_round;
  if (ngroups > 1 || (last != 0 && last < per_round / 2)) {
    // groups of the l-sum are the slowest index, so the workgroups running
    // together on one XCD sum the same subblocks l
    const int64_t lin = (bid & 7) * per_xcd + (bid >> 3);
    if (lin >= ntiles * ngroups) return;
    grp_l = lin / ntiles;
    by_groups(lin - grp_l * ntiles, pb.nI, nS, ti, ts);
  } else {
    // XCD x runs tiles [T0, T1) of the order; of those, a share of the border
    // tiles proportional to the count comes last
    const int64_t nIf = pb.M / L, nSf = pb.N / F::TN;
    const int64_t nF = nIf * nSf, nB = ntiles - nF;
    const int64_t x = bid & 7, k = bid >> 3;
    const int64_t T0 = min(x * per_xcd, ntiles), T1 = min((x + 1) * per_xcd, ntiles);
    const int64_t b0 = nB * T0 / ntiles, nb = nB * T1 / ntiles - b0;
    const int64_t f0 = T0 - b0, nf = (T1 - T0) - nb;
    if (k < nf) {
      by_groups(f0 + k, nIf, nSf, ti, ts);
    } else if (k < nf + nb) {
      // border tiles: the last slab column over the full tile rows, then the last tile row
      const int64_t t = b0 + (k - nf);
      const int64_t ncol = nS > nSf ? nIf : 0;
      if (t < ncol) { ti = t; ts = nS - 1; }
      else { ti = pb.nI - 1; ts = t - ncol; }
    } else {
      return;
    }
  }
  const int64_t tj = ts / SLABS;
  const int64_t l0 = grp_l * g.gsize;
  const int64_t nl = min(g.gsize, pb.nL - l0);
  F f(pb, A, B, sm, ti * L, ts * F::TN);
  f.kb = l0 * L;
  const tdgemm_pair *prs = g.pairs + (ti * pb.nJ + tj) * pb.nL + l0;
  const bool interior = (ti + 1) * L <= pb.M && (ts + 1) * F::TN <= pb.N;
  if (interior) f.template run<false>(prs, nl);
  else f.template run<true>(prs, nl);
  if (ngroups > 1) f.write_c(part + grp_l * pb.M * pb.N, pb.N);
  else f.write_c(C, pb.ldc);
}

// C = sum over the groups g (ascending, from zero) of their partial results.
// The partials are loaded eight groups at a time before they are added in
// order, so that a thread has eight loads in flight (few threads, many groups).
template <typename PT>
__global__ __launch_bounds__(256) void k_sum_groups(const PT *__restrict__ part, int64_t ngroups,
                                                    int64_t M, int64_t N, PT *__restrict__ C,
                                                    int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = M * N;
  if (e >= mn) return;
  PT total = (PT)0;
  int64_t q = 0;
  for (; q + 8 <= ngroups; q += 8) {
    PT v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(q + u) * mn + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) total = total + v[u];
  }
  for (; q < ngroups; ++q) total = total + part[q * mn + e];
  const int64_t r = e / N;
  C[r * ldc + (e - r * N)] = total;
}

// ---------------------------------------------------------------------------
template <typename IT, typename PT, int L, int FORM>
static hipError_t launch_fused_t(const GemmOperands &g, const void *A, const void *B, void *C,
                                 void *part, hipStream_t st) {
  typedef Fused<IT, PT, L, FORM, false, false> F0;
  const int64_t ntiles = g.pb.nI * g.pb.nJ * (L / F0::TN);
  const int64_t ngroups = (g.pb.nL + g.gsize - 1) / g.gsize;
  const int64_t per_xcd = (ntiles * ngroups + 7) / 8;
  const dim3 grid((unsigned)(per_xcd * 8));
  const dim3 block(F0::NT);
  const IT *a = (const IT *)A;
  const IT *b = (const IT *)B;
  PT *c = (PT *)C;
  PT *p = (PT *)part;
  if (!g.ta && !g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, false, false>), grid, block, 0, st, g, a, b, c, p, ntiles, ngroups, per_xcd);
  else if (g.ta && !g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, true, false>), grid, block, 0, st, g, a, b, c, p, ntiles, ngroups, per_xcd);
  else if (!g.ta && g.tb)
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, false, true>), grid, block, 0, st, g, a, b, c, p, ntiles, ngroups, per_xcd);
  else
    hipLaunchKernelGGL((k_fused<IT, PT, L, FORM, true, true>), grid, block, 0, st, g, a, b, c, p, ntiles, ngroups, per_xcd);
  if (ngroups > 1) {
    const int64_t n = g.pb.M * g.pb.N;
    hipLaunchKernelGGL((k_sum_groups<PT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, ngroups,
                       g.pb.M, g.pb.N, c, g.pb.ldc);
  }
  return hipGetLastError();
}

// Launch for one (input type, packing type, L): the form and the transposes
// are dispatched here; fused_*.hip instantiate it, one combination per file.
template <typename IT, typename PT, int L>
hipError_t launch_fused_il(const GemmOperands &g, const void *A, const void *B, void *C, void *part,
                           hipStream_t st) {
  return g.form == TDGEMM_SYM ? launch_fused_t<IT, PT, L, TDGEMM_SYM>(g, A, B, C, part, st)
                              : launch_fused_t<IT, PT, L, TDGEMM_ASYM>(g, A, B, C, part, st);
}

#define TDG_FUSED_INSTANCE(IT, PT, L)                                                         \
  template hipError_t launch_fused_il<IT, PT, L>(const GemmOperands &, const void *,        \
                                                 const void *, void *, void *, hipStream_t);

#define TDG_FUSED_EXTERN(IT, PT, L)                                                           \
  extern template hipError_t launch_fused_il<IT, PT, L>(const GemmOperands &, const void *, \
                                                        const void *, void *, void *, hipStream_t);

}  // namespace tdg
