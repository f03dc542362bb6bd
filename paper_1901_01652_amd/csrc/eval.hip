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
#include "mfma.hpp"

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

// FP32 input: Psi tiles on the FP32 matrix cores.  L and R^T are first copied to FP32 with
// the contraction padded to a multiple of 4.  A work-group owns a 128 (il) x 256 (ir) tile;
// blocks run il-block fastest, so the 8 XCDs each reuse one R^T chunk from L2 and keep their
// share of L resident.  Each wavefront covers 32 rows; per group of four 16-column tiles it
// first loads its X values (in flight together) and then forms the Psi tiles,
// accumulating (x - psi)^2 and x^2 in FP64.
constexpr int kRtM = 128, kRtN = 256;

__global__ __launch_bounds__(256) void pad_f32_kernel(const double* __restrict__ src, int64_t rows,
                                                      int RR, int RRp, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * RRp) return;
  const int64_t r = e / RRp;
  const int k = (int)(e - r * RRp);
  dst[e] = k < RR ? (float)src[r * RR + k] : 0.f;
}

__global__ __launch_bounds__(256, 3) void residual_mfma_kernel(const float* __restrict__ X,
                                                            int64_t IL, int64_t IR, int RRp,
                                                            const float* __restrict__ Lf,
                                                            const float* __restrict__ Rf,
                                                            int64_t nil, double* __restrict__ partial) {
  extern __shared__ float rsm[];
  __shared__ double red[16];
  const int ldk = RRp + 1;
  float* Ls = rsm;                 // kRtM x ldk
  float* Rs = rsm + kRtM * ldk;    // kRtN x ldk
  const int64_t ilb = blockIdx.x % nil, irb = blockIdx.x / nil;
  const int64_t il0 = ilb * kRtM, ir0 = irb * kRtN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c16 = lane & 15;
  {
    // 16-byte copies: thread t owns column group t % q4 of every (256 / q4)-th row
    const int q4 = RRp >> 2, k4 = tid % q4, rstep = 256 / q4;
    int r = tid / q4;
    if (r < rstep) {
      for (int rr = r; rr < kRtM + kRtN; rr += rstep) {
        const bool isL = rr < kRtM;
        const int64_t src_row = isL ? il0 + rr : ir0 + (rr - kRtM);
        const bool ok = src_row < (isL ? IL : IR);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok) v = *(const float4*)((isL ? Lf : Rf) + src_row * RRp + 4 * k4);
        float* d = rsm + rr * ldk + 4 * k4;  // Ls rows, then Rs rows
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
      }
    }
  }
  __syncthreads();
  double sres = 0.0, sx = 0.0;
  // this lane's 8 rows of X (clamped to a valid row; out-of-range rows are masked below)
  const float* xr[8];
  unsigned rowok = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t row = il0 + 32 * w + 16 * (q >> 2) + 4 * g + (q & 3);
    rowok |= (row < IL ? 1u : 0u) << q;
    xr[q] = X + (row < IL ? row : 0) * IR;
  }
#pragma unroll 1
  for (int jg = 0; jg < kRtN / 16; jg += 4) {
    float xv[2][4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // unconditional loads from clamped (valid) addresses, masked by a multiply afterwards
      // (a select lets the compiler sink each load into a branch with its own wait), so that
      // the 32 loads issue back to back
      const int64_t col = ir0 + 16 * (jg + j) + c16;
      const bool cok = col < IR;
      const int64_t colc = cok ? col : IR - 1;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float mk = (cok && ((rowok >> q) & 1u)) ? 1.f : 0.f;
        xv[q >> 2][j][q & 3] = xr[q][colc] * mk;  // clamped entries are finite tensor values
      }
    }
    // keep all 32 loads of the group ahead of the products (in flight together)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = t >> 2, j = t & 3;
      const float* a = Ls + (32 * w + 16 * i + c16) * ldk + g;
      const float* b = Rs + (16 * (jg + j) + c16) * ldk + g;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
      for (int k0 = 0; k0 < RRp; k0 += 4)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k0], b[k0], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double x = (double)xv[i][j][r];
        const double d = x - (double)acc[r];
        sres += d * d;
        sx += x * x;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // rows or columns beyond the tensor hold x = 0 and psi = 0 (zero L / R^T rows): no effect
  sres = block_sum(sres, red);
  sx = block_sum(sx, red);
  if (tid == 0) {
    partial[2 * blockIdx.x] = sres;
    partial[2 * blockIdx.x + 1] = sx;
  }
}

// The matrix-core residual keeps a (128 + 256) x (RR + 1) FP32 tile in LDS: RR <= 96.
static bool residual_mfma_ok(bool f32, int RR) { return f32 && ((RR + 3) & ~3) <= 96; }

int64_t residual_blocks(bool f32, int64_t IL, int64_t IR, int RR) {
  if (residual_mfma_ok(f32, RR)) return ((IL + kRtM - 1) / kRtM) * ((IR + kRtN - 1) / kRtN);
  const int64_t ir_tiles = (IR + 255) / 256;
  int64_t ilb = kResBlocks / ir_tiles;
  if (ilb < 1) ilb = 1;
  if (ilb > IL) ilb = IL;
  const int64_t il_per = (IL + ilb - 1) / ilb;
  return ir_tiles * ((IL + il_per - 1) / il_per);
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
                           const double* L, const double* RtT, double* partial, float* lr32,
                           double* out, hipStream_t s) {
  prof_begin("residual", s);
  unsigned blocks;
  if (residual_mfma_ok(f32, RR)) {
    const int RRp = (RR + 3) & ~3;
    float* Lf = lr32;
    float* Rf = lr32 + IL * RRp;
    hipLaunchKernelGGL(pad_f32_kernel, dim3((unsigned)((IL * RRp + 255) / 256)), dim3(256), 0, s, L,
                       IL, RR, RRp, Lf);
    hipLaunchKernelGGL(pad_f32_kernel, dim3((unsigned)((IR * RRp + 255) / 256)), dim3(256), 0, s,
                       RtT, IR, RR, RRp, Rf);
    const int64_t nil = (IL + kRtM - 1) / kRtM;
    blocks = (unsigned)residual_blocks(true, IL, IR, RR);
    const size_t lds = (size_t)(kRtM + kRtN) * (RRp + 1) * sizeof(float);
    hipError_t e = hipFuncSetAttribute((const void*)residual_mfma_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_mfma_kernel, dim3(blocks), dim3(256), lds, s, (const float*)X, IL,
                       IR, RRp, Lf, Rf, nil, partial);
  } else {
    const int64_t ir_tiles = (IR + 255) / 256;
    int64_t ilb = kResBlocks / ir_tiles;
    if (ilb < 1) ilb = 1;
    if (ilb > IL) ilb = IL;
    const int64_t il_per = (IL + ilb - 1) / ilb;
    blocks = (unsigned)residual_blocks(f32, IL, IR, RR);
    if (f32)
      hipLaunchKernelGGL((residual_kernel<float, false>), dim3(blocks), dim3(256), 0, s,
                         (const float*)X, IL, IR, RR, L, RtT, ir_tiles, il_per, partial);
    else if (RR <= kResRR)
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
