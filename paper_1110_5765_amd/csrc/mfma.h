// 16 x 16 x 4 matrix-core products for FP64 and FP32 on gfx950.
//
// Operand layout (both types): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]. Result: lane l, register r holds D[row(l, r)][l % 16].
// Measured on the target: the FP64 result row is l / 16 + 4 r, the FP32 one
// 4 (l / 16) + r; both accumulate exactly as a chain of fused multiply-adds
// over k = 0, 1, 2, 3 starting from the accumulator.
#pragma once

#include <hip/hip_runtime.h>

namespace tdg {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename PT> struct Mfma;

template <> struct Mfma<double> {
  typedef d4_t Acc;
  __device__ __forceinline__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ __forceinline__ static Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <> struct Mfma<float> {
  typedef f4_t Acc;
  __device__ __forceinline__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ __forceinline__ static Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

}  // namespace tdg
