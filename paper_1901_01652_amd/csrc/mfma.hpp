// Matrix-core helpers for gfx950: one 16x16 output tile of C = A * Bt^T with both operands
// stored in LDS with the contraction index contiguous (A row-major M x K, Bt row-major
// N x K).  Lane l of a wavefront owns row (l & 15) of the A slice and row (l & 15) of the
// Bt slice, contraction group (l >> 4); the accumulator holds C[4*(l>>4) + r][l & 15],
// r = 0..3.
//   bf16: v_mfma_f32_16x16x32_bf16, 8 contraction elements per lane (one 16-byte read)
//   fp32: v_mfma_f32_16x16x4_f32, 1 contraction element per lane
#pragma once
#include <hip/hip_runtime.h>

namespace rtr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// kdim: multiple of 32 (bf16) / 4 (fp32); operands zero-padded up to kdim.
__device__ __forceinline__ f32x4 tile_abt(const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                          int kdim, f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const __bf16* a = A + r * lda + g * 8;
  const __bf16* b = Bt + r * ldb + g * 8;
  for (int k = 0; k < kdim; k += 32) {
    const bf16x8 av = *(const bf16x8*)(a + k);
    const bf16x8 bv = *(const bf16x8*)(b + k);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ f32x4 tile_abt(const float* A, int lda, const float* Bt, int ldb,
                                          int kdim, f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const float* a = A + r * lda + g;
  const float* b = Bt + r * ldb + g;
  for (int k = 0; k < kdim; k += 4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], b[k], acc, 0, 0, 0);
  return acc;
}

// Element type of the LDS operands and the contraction granule for each arithmetic.
template <bool BF>
struct Mma;
template <>
struct Mma<true> {
  using T = __bf16;
  static constexpr int kStep = 32;
  static __device__ __forceinline__ __bf16 cvt(float v) { return (__bf16)v; }
};
template <>
struct Mma<false> {
  using T = float;
  static constexpr int kStep = 4;
  static __device__ __forceinline__ float cvt(float v) { return v; }
};

// FP64 matrix cores, v_mfma_f64_16x16x4_f64: lane l supplies A[l & 15][l >> 4] and
// B[l >> 4][l & 15]; the accumulator holds C[4 r + (l >> 4)][l & 15] for r = 0..3 (rows are
// interleaved across lane groups, unlike the FP32 and bf16 forms).
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace rtr
