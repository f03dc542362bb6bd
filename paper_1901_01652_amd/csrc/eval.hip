// Alg. 1 steps 10-12 (back-projection G_n = Z_n x_2 Q_n) and the Sec. 4 error measure
// ||X - Psi([G_n])||_F^2.
//
// The residual splits the modes into a left half (1..h) and a right half (h+1..N); the
// chain kernel forms L[il] = G_1(i_1)..G_h(i_h) and Rt[ir] = G_{h+1}(i_{h+1})..G_N(i_N)
// (stored transposed), so Psi at (il, ir) = Trace(L[il] Rt[ir]) is a dot product of length
// R_1 R_{h+1}.  A work-group walks a block of il for a fixed tile of ir; each thread keeps
// its Rt row in registers.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

__global__ __launch_bounds__(256) void backproject_kernel(const double* __restrict__ Z,
                                                          const double* __restrict__ Q, int Ra,
                                                          int K, int64_t In, int Rb,
                                                          double* __restrict__ G) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)Ra * In * Rb) return;
  const int b = (int)(p % Rb);
  const int64_t i = (p / Rb) % In;
  const int a = (int)(p / ((int64_t)Rb * In));
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += Q[i * K + k] * Z[((int64_t)a * K + k) * Rb + b];
  G[p] = s;
}

hipError_t launch_backproject(const double* Z, const double* Q, int Ra, int K, int64_t In,
                              int Rb, double* G, hipStream_t s) {
  const int64_t n = (int64_t)Ra * In * Rb;
  prof_begin("backproject", s);
  hipLaunchKernelGGL(backproject_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Z,
                     Q, Ra, K, In, Rb, G);
  prof_end(s);
  return hipGetLastError();
}

constexpr int kResRR = 64;      // register copy of an Rt row when R_1 R_{h+1} <= 64
constexpr int kResBlocks = 2048;

template <typename T, bool REG>
__global__ __launch_bounds__(256) void residual_kernel(const T* __restrict__ X, int64_t IL,
                                                       int64_t IR, int RR,
                                                       const double* __restrict__ L,
                                                       const double* __restrict__ RtT,
                                                       int64_t ir_tiles, int64_t il_per,
                                                       double* __restrict__ partial) {
  __shared__ double red[16];
  const int64_t tile = blockIdx.x % ir_tiles;
  const int64_t ilb = blockIdx.x / ir_tiles;
  const int64_t ir = tile * 256 + threadIdx.x;
  const int64_t il0 = ilb * il_per;
  const int64_t il1 = min(IL, il0 + il_per);
  double s_res = 0.0, s_x = 0.0;
  if (ir < IR) {
    double rt[REG ? kResRR : 1];
    if constexpr (REG) {
#pragma unroll
      for (int r = 0; r < kResRR; ++r) rt[r] = (r < RR) ? RtT[ir * RR + r] : 0.0;
    }
    for (int64_t il = il0; il < il1; ++il) {
      const double* l = L + il * RR;
      double psi = 0.0;
      if constexpr (REG) {
#pragma unroll
        for (int r = 0; r < kResRR; ++r)
          if (r < RR) psi += l[r] * rt[r];
      } else {
        for (int r = 0; r < RR; ++r) psi += l[r] * RtT[ir * RR + r];
      }
      const double x = (double)X[il * IR + ir];
      const double d = x - psi;
      s_res += d * d;
      s_x += x * x;
    }
  }
  s_res = block_sum(s_res, red);
  s_x = block_sum(s_x, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s_res;
    partial[2 * blockIdx.x + 1] = s_x;
  }
}

__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ partial,
                                                             int count, double* __restrict__ out) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

hipError_t launch_residual(bool f32, const void* X, int64_t IL, int64_t IR, int RR,
                           const double* L, const double* RtT, double* partial, double* out,
                           hipStream_t s) {
  const int64_t ir_tiles = (IR + 255) / 256;
  int64_t ilb = kResBlocks / ir_tiles;
  if (ilb < 1) ilb = 1;
  if (ilb > IL) ilb = IL;
  const int64_t il_per = (IL + ilb - 1) / ilb;
  ilb = (IL + il_per - 1) / il_per;
  const unsigned blocks = (unsigned)(ir_tiles * ilb);
  const bool reg = RR <= kResRR;
  prof_begin("residual", s);
  if (f32) {
    if (reg)
      hipLaunchKernelGGL((residual_kernel<float, true>), dim3(blocks), dim3(256), 0, s,
                         (const float*)X, IL, IR, RR, L, RtT, ir_tiles, il_per, partial);
    else
      hipLaunchKernelGGL((residual_kernel<float, false>), dim3(blocks), dim3(256), 0, s,
                         (const float*)X, IL, IR, RR, L, RtT, ir_tiles, il_per, partial);
  } else {
    if (reg)
      hipLaunchKernelGGL((residual_kernel<double, true>), dim3(blocks), dim3(256), 0, s,
                         (const double*)X, IL, IR, RR, L, RtT, ir_tiles, il_per, partial);
    else
      hipLaunchKernelGGL((residual_kernel<double, false>), dim3(blocks), dim3(256), 0, s,
                         (const double*)X, IL, IR, RR, L, RtT, ir_tiles, il_per, partial);
  }
  hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, s, partial, (int)blocks, out);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
