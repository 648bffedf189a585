/*
 * tdgemm.h -- throughput-distortion GEMM for AMD MI355X (gfx950).
 *
 * C = A B computed by the method of Anastasia & Andreopoulos, "Throughput-
 * Distortion Computation of Generic Matrix Multiplication": per-block adaptive
 * companding and rounding of A and B (Sec. 3.A, eq. 3), packing of W rounded
 * operands into one floating-point word in the symmetric (Sec. 3.B, eqs. 6-7)
 * or asymmetric (Sec. 3.C, eq. 11) form, the product of the packed L x L
 * subblocks (eqs. 8, 12), unpacking (eqs. 9-10, 13-14) and reverse companding
 * (eq. 5), with the companders and packings chosen per subblock pair by the
 * distortion control of Sec. 5.B and Sec. 6.
 *
 * Conventions shared by every entry point:
 *  - A, B, C and all buffers named "device" are device pointers owned by the
 *    caller; the library never allocates, frees or retains device memory.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Calls enqueue work on it and return without synchronising, except
 *    tdgemm_plan_export and tdgemm_calibrate, which say so.
 *  - Matrices are row-major. With trans_a = 0, A is M x K with leading
 *    dimension lda >= K; with trans_a = 1 the caller stores A^T (K x M,
 *    lda >= M). Likewise B (K x N, or N x K with trans_b). C is M x N, ldc >= N.
 *  - Argument and shape errors are detected on the host before anything is
 *    launched; the call then returns an error status and enqueues nothing.
 *    HIP launch errors return TDGEMM_E_HIP. Nothing throws across the ABI.
 *  - Subblock pairs (A_il, B_lj) are numbered pair = (i * nJ + j) * nL + l with
 *    nI = ceil(M/L), nL = ceil(K/L), nJ = ceil(N/L): inner kernel major, l fastest.
 *  - Per-pair staging buffers hold one L x L slot of `prec` elements per pair,
 *    row-major; packed blocks use the leading rows/columns of their slot.
 */
#ifndef TDGEMM_H
#define TDGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDGEMM_OK = 0,
  TDGEMM_E_ARG = -1,          /* invalid argument or shape */
  TDGEMM_E_UNSUPPORTED = -2,  /* valid but not implemented (e.g. L = 80) */
  TDGEMM_E_WORKSPACE = -3,    /* workspace missing or too small */
  TDGEMM_E_CALIB = -4,        /* calibration table missing or malformed */
  TDGEMM_E_HIP = -5           /* a HIP runtime call failed */
} tdgemm_status;

enum { TDGEMM_F64 = 0, TDGEMM_F32 = 1,                        /* element types */
       TDGEMM_I8 = 2, TDGEMM_E4M3 = 3 };                       /* block-scaled forms (prec only) */
enum { TDGEMM_SYM = 1, TDGEMM_ASYM = 2 };                      /* packing forms */
enum { TDGEMM_CTRL_SNR = 0, TDGEMM_CTRL_FIXED = 1, TDGEMM_CTRL_SEPARABLE = 2, TDGEMM_CTRL_ACCEL = 3,
       TDGEMM_CTRL_TARGET = 4 };

typedef struct {
  int64_t M, N, K;
  int64_t lda, ldb, ldc;       /* L * lda and L * ldb times the element size of
                                 in_dtype must be below 2^30 bytes
                                 (TDGEMM_E_UNSUPPORTED otherwise) */
  int32_t trans_a, trans_b;   /* 0 or 1, see conventions */
  int32_t in_dtype;           /* TDGEMM_F64 or TDGEMM_F32: element type of A and B */
  int32_t prec;               /* TDGEMM_F64 or TDGEMM_F32: arithmetic of the packed path
                                 (companding, packing, product, unpacking, reverse
                                 companding) and element type of C. F32 packing of
                                 F64 inputs is not supported.
                                 TDGEMM_I8 / TDGEMM_E4M3: the block-scaled form (Remark 1):
                                 no packing; the separable rounded operands [[c x]] (INT8,
                                 |.| <= sep_q <= 127) or E4M3FN(c x) (OCP FP8, sep_q <= 448)
                                 of every block are multiplied on the INT8 / FP8 matrix
                                 cores per pair and C (float32) accumulates
                                 fma(float(r), float(1/(c_A c_B)), C) over l ascending.
                                 Requires ctrl = SEPARABLE, fixed_w = 1 and L = 128. */
  int32_t L;                  /* inner-kernel size, eq. (1): 64, 96 or 128. The packings W
                                 must divide L: {1, 2, 4} at L = 64 and 128, {1, 2, 3, 4}
                                 at L = 96 (the double-precision set of Sec. 7) */
  int32_t form;               /* TDGEMM_SYM or TDGEMM_ASYM */
  int32_t ctrl;               /* TDGEMM_CTRL_*:
                                 SNR: Sec. 5.B / Sec. 6 control to snr_db per inner kernel;
                                 FIXED: every pair at packing fixed_w and range fixed_rmax
                                        with the eq. (26) companders;
                                 SEPARABLE: every pair at packing fixed_w with per-block
                                        companders c = sep_q / max|block| (Sec. 3.A);
                                 ACCEL: the SNR-mode options pruned under the throughput
                                        constraint F_kernel = accel (Sec. 6);
                                 TARGET: every pair at packing fixed_w and range fixed_rmax
                                        with the Prop. 3 companders (eq. 22, the root with
                                        c_A >= c_A*) reaching the expected subblock SNR
                                        snr_db, s(R_max, W) read from the calibration table
                                        at the smallest grid R >= fixed_rmax; where eq. (25)
                                        fails (snr_db beyond what fixed_rmax allows) the
                                        eq. (26) companders, the highest SNR at fixed_rmax. */
  uint32_t w_allowed;         /* SNR / ACCEL: bit w set => packing W = w allowed; bit 1
                                 (W = 1, native arithmetic) must be set; W in {1, 2, 4}, or
                                 any of {1, 2, 3, 4} at L = 96 */
  int32_t fixed_w;            /* FIXED / SEPARABLE / TARGET: W in {1, 2, 4}, or {1, 2, 3, 4}
                                 at L = 96 */
  double snr_db;              /* SNR mode: S_kernel(i, j) in dB for every inner kernel
                                 (Sec. 6); +inf requests native precision everywhere.
                                 TARGET: the expected subblock SNR in dB (not -inf; +inf
                                 asks for the highest fixed_rmax allows) */
  double fixed_rmax;          /* FIXED / TARGET: R_max of eqs. (17), (24) */
  double sep_q;               /* SEPARABLE: integer range Q >= 1 of the rounded operands */
  double u_safe;              /* eq. (15) safety term, normally 50 */
  double accel;               /* ACCEL: F_kernel in [0, 1]. Each inner kernel keeps saving at
                                 least accel * nL * (1 - 1/W_max) of the W = 1 MFMA work,
                                 sum_l (1 - 1/W_l) (or, with accel_units, of the measured
                                 time); with W in {1, 2} it is the fraction of
                                 subblock products that stay packed. Starting from W_max
                                 everywhere, the pair with the largest D (lowest l on ties)
                                 drops to the next allowed W while the constraint still holds
                                 afterwards and that D is positive. */
  const double *tile_target;  /* SNR / ACCEL, optional (NULL: snr_db or accel for every inner
                                 kernel): host array of nI x nJ targets, row-major by inner-kernel
                                 row i, one per inner kernel R_ij (Sec. 6): S_kernel(i, j) in dB
                                 (SNR; not NaN, +inf = native precision), F_kernel(i, j) in
                                 [0, 1] (ACCEL), or the expected subblock SNR in dB of the
                                 pairs of R_ij (TARGET; not NaN or -inf). nI = ceil(M / L), nJ = ceil(N / L). Read during
                                 tdgemm_plan only, which then synchronises its stream once. Must
                                 be NULL in the other control modes. */
  int32_t k_split;            /* evaluation order of the l-sum of eq. (2): 0 or 1 = one
                                 ascending sum per inner kernel; k > 1 = groups of
                                 s = ceil(nL / k) consecutive subblocks, each summed from zero
                                 in ascending l by its own workgroup of the fused kernel, then
                                 the ceil(nL / s) group sums added in ascending order to zero
                                 (more workgroups when M and N give few inner kernels). The
                                 workspace then holds ceil(nL / s) partial M x N results of
                                 prec. Not for the block-scaled forms (TDGEMM_E_UNSUPPORTED). */
  int32_t accel_units[5];     /* ACCEL, optional: the time a pair saves at packing W against
                                 W = 1, accel_units[W] for W = 2..4, in integer units (Sec. 5.B
                                 keeps the acceleration F_W of every packing, measured off-line
                                 on the target: units = round(scale (1 - 1/F_W)), scale <= 2^20).
                                 Entries 0 and 1 must be 0, the others in [0, 2^20]. All zero:
                                 nominal MFMA work, 12 - 12/W twelfths of a W = 1 product.
                                 The constraint then reads sum_l units[W_l] >=
                                 accel * nL * units[W_max]. Ignored in the other modes. */
} tdgemm_desc;

/* Representation-noise table s(R_max, W) of Sec. 4.B (eq. 18), device memory:
 * r[n_r] strictly ascending R values shared by all W (n_r <= 512); s[3 * n_r] the RMSE in index
 * units for W = 2 (row 0), 3 (row 1) and 4 (row 2); +inf marks an unusable
 * point. Read by the plan's kernels only: keep it alive until the stream has
 * run them. */
typedef struct {
  int32_t n_r;
  const double *r;
  const double *s;
} tdgemm_calib;

/* Statistics of one block over its valid elements (Sec. 3, Sec. 5.B):
 * sigma = sqrt(sumsq / n); sumsq is the sum of squares rounded once. */
typedef struct {
  double mn, mx, sumsq;
  int64_t n;
} tdgemm_block_stats;

/* One pair's settings (Sec. 5.B option record after the Sec. 6 pruning). */
typedef struct {
  double c_a, c_b;            /* companders, eq. (26) (or Q / max|X| when separable) */
  double inv;                 /* 1 / (c_a c_b), eq. (5) */
  double d;                   /* expected noise power D_W, eq. (21) */
  double r_max;               /* R_max* */
  double s_rep;               /* s(R_max*, W) */
  double q_a, q_b;            /* [[c max|X|]]: bounds of the rounded operands */
  int32_t w;                  /* packing W (1 = native floating point) */
  int32_t p;                  /* z = 2^-p, eq. (15) */
} tdgemm_pair;

typedef struct tdgemm_plan_s *tdgemm_plan_t;   /* opaque, host memory */

/* Bytes of device workspace tdgemm_plan needs for this descriptor (block
 * statistics, pair records, inner-kernel budgets). 0 if the descriptor is
 * invalid. */
size_t tdgemm_workspace_size(const tdgemm_desc *desc);

/* Sec. 5.B and Sec. 6: per-block statistics of A and B (min, max, sum of
 * squares), per-pair options for every allowed W (eq. 26 companders at the R_max
 * minimising the eq. 27 noise over the calibrated grid, z from eq. 15, D_W from
 * eq. 21) and, per inner kernel, top-down pruning to the SNR budget.
 * calib is also required in TARGET mode (s(R_max, W) of eq. 23).
 * A, B: device inputs (described by desc). calib: required in SNR mode, else
 * may be NULL. ws: device workspace of ws_bytes >= tdgemm_workspace_size(desc);
 * it holds the plan and must outlive it. On success *out receives a new plan
 * (host object, release with tdgemm_plan_destroy). Enqueues the statistics and
 * plan kernels on stream. */
tdgemm_status tdgemm_plan(const tdgemm_desc *desc, const void *A, const void *B,
                          const tdgemm_calib *calib, void *ws, size_t ws_bytes,
                          void *stream, tdgemm_plan_t *out);

/* Eq. (3): qA[pair] = [[c_a A_il]], qB[pair] = [[c_b B_lj]] per pair (round half
 * to even, in prec; out-of-range elements 0). W = 1 pairs copy the block
 * unrounded. qA, qB: device, n_pairs * L * L elements of prec each.
 * Block-scaled forms (prec I8 / E4M3): one byte per element of every block,
 * shared by all pairs: qA is (nI L) x (nL L) bytes, row m of A with K
 * contiguous; qB is (nJ L) x (nL L) bytes, column n of B with K contiguous
 * (B^T); INT8 two's complement or E4M3FN codes; padding is 0. */
tdgemm_status tdgemm_compand(tdgemm_plan_t plan, const void *A, const void *B,
                             void *qA, void *qB, void *stream);

/* Packing. Symmetric (eqs. 6-7): pA[pair] is L x L/W with W consecutive
 * columns of qA per word (weights z^i), pB[pair] is L/W x L with W consecutive
 * rows of qB per word (weights z^-i). Asymmetric (eq. 11): pA[pair] is L/W x L
 * with W consecutive rows of qA per word (weights z^i); pB[pair] = qB. Words are
 * evaluated by Horner's rule from the highest slot. W = 1 pairs copy.
 * Buffers: device, n_pairs * L * L elements of prec each. The block-scaled
 * forms pack nothing: TDGEMM_E_UNSUPPORTED. */
tdgemm_status tdgemm_pack(tdgemm_plan_t plan, const void *qA, const void *qB,
                          void *pA, void *pB, void *stream);

/* Packed product (eqs. 8, 12) on the matrix cores, each output accumulated over
 * the packed index in ascending order.
 * fused = 0: a = pA, b = pB (as written by tdgemm_pack); out = Rbar, device,
 *            n_pairs * L * L elements of prec (L x L symmetric, L/W x L asymmetric).
 * fused = 1: a = A, b = B (as given to tdgemm_plan); out = C. One kernel runs
 *            every stage per pair -- compand, pack, packed product, unpack,
 *            reverse companding -- and accumulates C over l ascending.
 * Block-scaled forms: a = qA, b = qB as written by tdgemm_compand. fused = 0:
 * out = the per-pair products r, n_pairs * L * L elements (int32 for I8, exact;
 * float32 for E4M3, the matrix cores' float32 sums), row-major per pair.
 * fused = 1: out = C (float32, ldc), C = fma(float(r), float(1/(c_A c_B)), C)
 * for l ascending from C = 0 (one rounding per pair). */
tdgemm_status tdgemm_gemm(tdgemm_plan_t plan, const void *a, const void *b, void *out,
                          int fused, void *stream);

/* Unpacking (eqs. 9-10 or 13-14) of every pair's Rbar into integers, then
 * reverse companding (eq. 5) and the l-sum of eq. (2), l ascending:
 * C_ij = sum_l r_l * inv_l (W = 1 pairs add their native product).
 * r_int: optional device buffer (NULL to skip) receiving the unpacked integers,
 * n_pairs * L * L elements of prec. C: device output (overwritten), or NULL
 * when only r_int is wanted (at least one of the two must be given).
 * Block-scaled forms: Rbar = the per-pair products of tdgemm_gemm(fused = 0);
 * r_int must be NULL; C (float32) as for fused = 1. */
tdgemm_status tdgemm_unpack(tdgemm_plan_t plan, const void *Rbar, void *r_int, void *C,
                            void *stream);

/* Summary of a plan (Sec. 6 and Prop. 3). Synchronises the stream the plan was
 * made on, then reads its statistics and pair records. Any pointer may be NULL.
 *  pred_snr_db  predicted output SNR of C in dB: 10 log10 of the sum over all
 *               pairs of the signal power L_eff sigma_a^2 sigma_b^2 (block RMS
 *               values, L_eff the valid inner extent) over the sum of their
 *               expected noise powers D (eq. 21); +inf when every D is 0 (all
 *               native, or an empty product). Block-scaled forms: D is the noise
 *               of rounding to the integer grid of range sep_q (eq. 19), which
 *               fits INT8; E4M3 rounds more coarsely (3 mantissa bits), so its
 *               prediction is optimistic.
 *  w_hist       5 counters: w_hist[W] = pairs at packing W (W = 1..4); w_hist[0] = 0.
 *  n_short      TARGET control: pairs at W >= 2 whose expected SNR (signal / D)
 *               is below their target (eq. 25 fails there and the eq. (26)
 *               companders, the best at fixed_rmax, are used); 0 otherwise.
 * Errors: TDGEMM_E_ARG for a NULL plan, TDGEMM_E_HIP if the copy fails. */
tdgemm_status tdgemm_plan_query(tdgemm_plan_t plan, double *pred_snr_db, int64_t *w_hist,
                                int64_t *n_short);

/* Copy the plan's statistics and records to host memory. Any pointer may be
 * NULL. Sizes: stats_a nI * nL, stats_b nL * nJ, pairs n_pairs, budgets nI * nJ
 * (D_kernel per inner kernel, SNR mode; 0 otherwise). Synchronises the stream
 * the plan was made on. */
tdgemm_status tdgemm_plan_export(tdgemm_plan_t plan, tdgemm_block_stats *stats_a,
                                 tdgemm_block_stats *stats_b, tdgemm_pair *pairs,
                                 double *budgets);

/* Grid of the plan: nI, nL, nJ and n_pairs = nI * nL * nJ. */
tdgemm_status tdgemm_plan_dims(tdgemm_plan_t plan, int64_t *nI, int64_t *nL, int64_t *nJ,
                               int64_t *n_pairs);

tdgemm_status tdgemm_plan_destroy(tdgemm_plan_t plan);

/* Representation-noise measurement of Sec. 4.B (eq. 18) on the GPU path, at
 * packing W > 1 (a packing L supports, see tdgemm_desc.L): for each integer range q[t] (host, n_q values >= 1) the inputs are integers
 * uniform on {-q..q}, obtained from the uniform [0, 1) draws u_a, u_b (device,
 * n_inst * L * L each) as floor(u (2q + 1)) - q; c_A = c_B = 1; R_max = L q^2;
 * z from eq. (15). The packed product of each instance is unpacked and compared
 * with the exact product. Outputs (host, n_q each): r_out = R_max, m_out = mean
 * error, s_out = RMSE (index units; +inf where non-finite). ws: device
 * workspace of at least tdgemm_calibrate_workspace_size(L, n_inst) bytes.
 * Synchronises the stream. */
size_t tdgemm_calibrate_workspace_size(int32_t L, int32_t n_inst);
tdgemm_status tdgemm_calibrate(int32_t L, int32_t W, int32_t form, int32_t prec,
                               const double *q, int32_t n_q, const double *u_a,
                               const double *u_b, int32_t n_inst, double u_safe,
                               double *r_out, double *m_out, double *s_out, void *ws,
                               size_t ws_bytes, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): tdgemm_plan followed by
 * tdgemm_gemm(fused = 1) with the plan's workspace in a static device array of
 * TDGEMM_NOALLOC_MAX_BYTES bytes per GPU instead of a caller workspace. It
 * allocates neither device nor host memory and does not synchronise.
 * desc, A, B, calib: as for tdgemm_plan; C: device output as for
 * tdgemm_gemm(fused = 1). stream must belong to the current device.
 * Errors (checked on the host before anything is enqueued):
 *   TDGEMM_E_WORKSPACE    tdgemm_workspace_size(desc) > TDGEMM_NOALLOC_MAX_BYTES;
 *   TDGEMM_E_UNSUPPORTED  desc->tile_target != NULL, or a block-scaled form;
 *   otherwise those of tdgemm_plan and tdgemm_gemm.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap on one GPU (on other streams or from other host
 * threads) race and give wrong results. */
#define TDGEMM_NOALLOC_MAX_BYTES ((size_t)32 << 20)
tdgemm_status tdgemm_matmul_noalloc(const tdgemm_desc *desc, const void *A, const void *B,
                                    const tdgemm_calib *calib, void *C, void *stream);

/* Human-readable name of a status code (static storage). */
const char *tdgemm_status_string(tdgemm_status status);

#ifdef __cplusplus
}
#endif

#endif /* TDGEMM_H */
