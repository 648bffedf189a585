// Launch wrappers of the tdgemm kernels (host side, namespace tdg).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace tdg {

// Statistics of every block of A and B, and (table != nullptr) the
// non-dominated calibration table, in one launch.
struct StatsArgs {
  const void *A, *B;
  int64_t M, N, K, lda, ldb;
  int ta, tb;
  int64_t nI, nL, nJ;
  tdgemm_block_stats *stats_a;   // [nI][nL]
  tdgemm_block_stats *stats_b;   // [nL][nJ]
  const double *calib_r, *calib_s;
  int n_r;
  PlanTable *table;
};

struct PlanLaunch {
  Problem pb;
  const tdgemm_block_stats *stats_a;
  const tdgemm_block_stats *stats_b;
  tdgemm_pair *pairs;
  double *budget;
  const double *calib_r;
  const double *calib_s;
  const PlanTable *table;
  int n_r;
  int ctrl;
  int n_opt;
  int w_desc[4];
  int fixed_w;
  int block_scaled;                    // INT8 / FP8 form: separable records with W = 1
  double fixed_rmax, sep_q, u_safe, snr_lin;
  double accel;                        // throughput constraint F_kernel (ACCEL control)
  int units[5];                        // ACCEL: saved work per pair at packing W (units[1] = 0)
  const double *tile;                  // [nI][nJ] per inner kernel: 10^(-S/10) (SNR),
                                       // F_kernel (ACCEL) or 10^(S/10) (TARGET); nullptr:
                                       // snr_lin / accel / tgt_pow everywhere
  double tgt_pow;                      // TARGET: 10^(S/10) of the expected subblock SNR
};

// Operands of the packed path (all device pointers).
struct GemmOperands {
  Problem pb;
  int in_dtype, prec, form;
  bool ta, tb;
  const tdgemm_pair *pairs;   // [n_pairs]
  int64_t gsize;              // subblocks per group of the l-sum (nL: one group)
};

hipError_t launch_stats(const StatsArgs &a, int dtype, int L, hipStream_t st);
hipError_t launch_plan(const PlanLaunch &p, hipStream_t st);

// staged path
hipError_t launch_compand(const GemmOperands &g, const void *A, const void *B, void *qA, void *qB,
                          hipStream_t st);
hipError_t launch_pack(const GemmOperands &g, const void *qA, const void *qB, void *pA, void *pB,
                       hipStream_t st);
hipError_t launch_packed_product(const GemmOperands &g, const void *pA, const void *pB, void *Rbar,
                                 hipStream_t st);
hipError_t launch_unpack(const GemmOperands &g, const void *Rbar, void *r_int, void *C,
                         hipStream_t st);

// fused path
// part: partial results of the groups (ngroups x M x N of prec) when gsize < nL, else unused.
hipError_t launch_fused(const GemmOperands &g, const void *A, const void *B, void *C, void *part,
                        hipStream_t st);

// Block-scaled INT8 / FP8 form (L = 128)
struct Quant8Args {
  const void *A, *B;
  int64_t M, N, K, lda, ldb;
  int ta, tb;
  int64_t nI, nL, nJ;
  int64_t Kp;                          // nL * 128: row length of qA and qB in bytes
  const tdgemm_block_stats *stats_a, *stats_b;
  double q;                            // Q of the block scales c = Q / max|X|
  uint8_t *qA, *qB;                    // [nI*128][Kp], [nJ*128][Kp]
};

struct Gemm8Args {
  const uint8_t *qA, *qB;
  int64_t Kp, nI, nL, nJ, M, N, ldc;
  const tdgemm_pair *pairs;
  const void *in;                      // staged products (k_scale_sum8)
  void *out;                           // C (float32) or staged products
};

hipError_t launch_quant8(const Quant8Args &a, int in_dtype, int fmt, hipStream_t st);
hipError_t launch_gemm8(const Gemm8Args &a, int fmt, bool staged, hipStream_t st);
hipError_t launch_scale_sum8(const Gemm8Args &a, int fmt, hipStream_t st);

hipError_t launch_fill_zero(void *C, int prec, int64_t M, int64_t N, int64_t ldc, hipStream_t st);

// calibration helpers (integer inputs from uniforms; error moments)
hipError_t launch_int_inputs(const double *u, int64_t n, double q, int prec, void *out,
                             hipStream_t st);
hipError_t launch_error_moments(const void *r, const double *ref, int prec, int64_t n,
                                double *out2, hipStream_t st);

}  // namespace tdg
