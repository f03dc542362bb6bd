// Matrix-core helpers for gfx950: one 16x16 output tile of C = A * Bt^T with both operands
// stored in LDS with the contraction index contiguous (A row-major M x K, Bt row-major
// N x K).  Lane l of a wavefront owns row (l & 15) of the A slice and row (l & 15) of the
// Bt slice, contraction group (l >> 4); the accumulator holds C[4*(l>>4) + r][l & 15],
// r = 0..3.
//   bf16: v_mfma_f32_16x16x32_bf16, 8 contraction elements per lane (one 16-byte read)
//   fp8:  v_mfma_f32_16x16x32_fp8_fp8 (OCP e4m3), 8 contraction elements per lane (8 bytes)
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

// fp8 e4m3 operands: 8 per lane packed in 64 bits.  kdim: multiple of 32.
__device__ __forceinline__ f32x4 tile_abt(const unsigned char* A, int lda, const unsigned char* Bt,
                                          int ldb, int kdim, f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const unsigned char* a = A + r * lda + g * 8;
  const unsigned char* b = Bt + r * ldb + g * 8;
  for (int k = 0; k < kdim; k += 32) {
    const long av = *(const long*)(a + k);
    const long bv = *(const long*)(b + k);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// Element type of the LDS operands, the contraction granule and the 8-element matrix-core
// step for each arithmetic: 0 FP32, 1 bf16, 2 fp8 (OCP e4m3; inputs clamped to +-448, the
// largest finite value, before rounding).
template <int PR>
struct Mma;
template <>
struct Mma<1> {
  using T = __bf16;
  using V8 = bf16x8;
  static constexpr int kStep = 32;
  static __device__ __forceinline__ __bf16 cvt(float v) { return (__bf16)v; }
  static __device__ __forceinline__ f32x4 mma8(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<2> {
  using T = unsigned char;
  using V8 = long;
  static constexpr int kStep = 32;
  static __device__ __forceinline__ unsigned char cvt(float v) {
    const float c = fminf(fmaxf(v, -448.f), 448.f);
    return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(c, 0.f, 0, false) & 0xFF);
  }
  static __device__ __forceinline__ f32x4 mma8(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<0> {
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
