/* Dot products as fused multiply-add chains (oracle; test infrastructure only).
 *
 * The packed products of eqs. (8) and (12) are ordinary matrix products run
 * "in the function's native representation". Their rounding depends on the
 * order of accumulation; the oracle fixes the plainest one: each output is
 * acc = 0; for k = 0, 1, ..., K-1: acc = fma(a[i][k], b[k][j], acc),
 * i.e. one correctly rounded fused multiply-add per term, in ascending k.
 * Built with -ffp-contract=off; fma()/fmaf() are C99's correctly rounded
 * fused operations.
 */
#include <math.h>
#include <stdint.h>

void oracle_fma_matmul_f64(const double *a, const double *b, double *c,
                           int64_t m, int64_t k, int64_t n) {
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int64_t t = 0; t < k; ++t) acc = fma(a[i * k + t], b[t * n + j], acc);
      c[i * n + j] = acc;
    }
}

void oracle_fma_matmul_f32(const float *a, const float *b, float *c,
                           int64_t m, int64_t k, int64_t n) {
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      float acc = 0.0f;
      for (int64_t t = 0; t < k; ++t) acc = fmaf(a[i * k + t], b[t * n + j], acc);
      c[i * n + j] = acc;
    }
}

/* Batched form: nb independent products, a[nb][m][k], b[nb][k][n], c[nb][m][n]. */
void oracle_fma_matmul_batched_f64(const double *a, const double *b, double *c,
                                   int64_t nb, int64_t m, int64_t k, int64_t n) {
  for (int64_t q = 0; q < nb; ++q)
    oracle_fma_matmul_f64(a + q * m * k, b + q * k * n, c + q * m * n, m, k, n);
}

void oracle_fma_matmul_batched_f32(const float *a, const float *b, float *c,
                                   int64_t nb, int64_t m, int64_t k, int64_t n) {
  for (int64_t q = 0; q < nb; ++q)
    oracle_fma_matmul_f32(a + q * m * k, b + q * k * n, c + q * m * n, m, k, n);
}
