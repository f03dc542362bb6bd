// Device-side helpers shared by the gfx950 kernels: Philox4x32-10, Box-Muller, bf16
// rounding, wavefront/block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtr.h"

namespace rtr {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds; each round multiplies
// counter words 0 and 2 by M0, M1 into 64-bit products and mixes in the key, which is
// advanced by the Weyl constants between rounds.
// ---------------------------------------------------------------------------------------
struct Ctr4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Ctr4 philox4x32_10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit product per word (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = Ctr4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Words of Philox call ``call`` of stream (seed, stream, tensor_id).
__device__ __forceinline__ Ctr4 philox_call(uint64_t seed, uint32_t stream, uint32_t tid,
                                            uint64_t call) {
  return philox4x32_10(Ctr4{(uint32_t)call, (uint32_t)(call >> 32), stream, tid},
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Box-Muller (1958) in FP64: u = (w + 1/2) 2^-32, r = sqrt(-2 ln u_a), theta = 2 pi u_b.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1) {
  const double ua = ((double)wa + 0.5) * 0x1p-32;
  const double ub = ((double)wb + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(ua));
  const double t = 6.283185307179586 * ub;
  double s, c;
  sincos(t, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// Box-Muller in FP32 on the transcendental unit: v_log_f32 is log2, v_sin/v_cos take the
// angle in revolutions, so theta = 2 pi u_b needs no multiply.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float ua = fmaf((float)wa, 0x1p-32f, 0x1p-33f);
  const float ub = fmaf((float)wb, 0x1p-32f, 0x1p-33f);
  const float r = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = r * __builtin_amdgcn_cosf(ub);
  z1 = r * __builtin_amdgcn_sinf(ub);
}

// Four consecutive stream elements 4*call .. 4*call+3.
template <typename T>
__device__ __forceinline__ void normals4(uint64_t seed, uint32_t stream, uint32_t tid,
                                         uint64_t call, T z[4]) {
  const Ctr4 w = philox_call(seed, stream, tid, call);
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}

// float -> bf16 -> float, round to nearest even (inputs are finite).
__device__ __forceinline__ float bf16_round(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// ---------------------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over the block; every thread gets the result.  ``scratch`` holds >= 16 T.
template <typename T>
__device__ T block_sum(T v, T* scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  return s;
}

// Work lists: job j owns grid blocks [block_start[j], block_start[j + 1]); the job of block b
// by binary search (block_start ascending, block_start[0] = 0).
__device__ __forceinline__ int find_job(const int64_t* __restrict__ block_start, int njobs,
                                        int64_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (block_start[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace rtr
