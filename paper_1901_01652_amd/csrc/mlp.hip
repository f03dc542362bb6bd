// Learned warm start for TR-ALS: a multilayer perceptron from the normalised projected
// tensor P~ = P / ||P|| to the packed initial cores, trained on ||P~ - Psi(Z)||^2 (Psi as in
// Eq. (1)).  Kernels:
//   gemm_kernel       C = op(A) op(B) on the matrix cores (bf16 operands rounded at the LDS
//                     stage, or FP32), FP32 accumulation, split over the contraction into
//                     per-slice partials;
//   epilogue_kernel   sum of the slices (fixed order) + bias + ReLU, or times the ReLU mask;
//   colsum_kernel     bias gradients;
//   tr_loss4_kernel   per sample: Psi of the four predicted cores, the residual, the loss and
//                     its gradient with respect to the cores (one work-group per sample);
//   adam_kernel       Adam update of one parameter array.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

namespace {
constexpr int kBM = 64, kBN = 64, kBK = 32;
}

template <bool BF>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  using T = typename Mma<BF>::T;
  constexpr int LD = BF ? kBK + 8 : kBK + 4;
  __shared__ __align__(16) T As[kBM * LD];
  __shared__ __align__(16) T Bs[kBN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int64_t kbeg = (int64_t)blockIdx.z * g.kslice;
  const int64_t kend = min((int64_t)g.K, kbeg + g.kslice);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool a_krow = g.sak == 1;  // A contiguous along k
  const bool b_kcol = g.sbk == 1;  // B contiguous along k
  for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
    for (int e = tid; e < kBM * kBK; e += 256) {
      int m, k;
      if (a_krow) {
        m = e / kBK;
        k = e % kBK;
      } else {
        m = e % kBM;
        k = e / kBM;
      }
      const int64_t gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < g.M && gk < kend) v = g.A[gm * g.sam + gk * g.sak];
      As[m * LD + k] = Mma<BF>::cvt(v);
    }
    for (int e = tid; e < kBN * kBK; e += 256) {
      int n, k;
      if (b_kcol) {
        n = e / kBK;
        k = e % kBK;
      } else {
        n = e % kBN;
        k = e / kBN;
      }
      const int64_t gn = n0 + n, gk = k0 + k;
      float v = 0.f;
      if (gn < g.N && gk < kend) v = g.B[gk * g.sbk + gn * g.sbn];
      Bs[n * LD + k] = Mma<BF>::cvt(v);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = tile_abt(As + (wm * 32 + 16 * i) * LD, LD, Bs + (wn * 32 + 16 * j) * LD, LD,
                             kBK, acc[i][j]);
    __syncthreads();
  }
  float* C = g.part + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * 32 + 16 * i + 4 * (lane >> 4) + r;
        const int64_t col = n0 + wn * 32 + 16 * j + (lane & 15);
        if (row < g.M && col < g.N) C[row * g.N + col] = acc[i][j][r];
      }
}

// out[m, n] = act(sum_z part[z, m, n] + bias[n]) (mode 0: none, 1: ReLU), or
// sum_z part[z, m, n] * (mask[m, n] > 0) (mode 2).
__global__ __launch_bounds__(256) void epilogue_kernel(const float* __restrict__ part,
                                                       int slices, int64_t M, int64_t N,
                                                       const float* __restrict__ bias,
                                                       const float* __restrict__ mask, int mode,
                                                       float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  float s = 0.f;
  for (int z = 0; z < slices; ++z) s += part[(int64_t)z * M * N + e];
  if (mode == 2) {
    out[e] = mask[e] > 0.f ? s : 0.f;
    return;
  }
  if (bias) s += bias[e % N];
  out[e] = (mode == 1) ? fmaxf(s, 0.f) : s;
}

__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ G, int64_t M,
                                                     int64_t N, float* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t m = 0; m < M; ++m) s += G[m * N + n];
  out[n] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ w,
                                                   const float* __restrict__ gr,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float omb1, float omb2, float eps, float c1,
                                                   float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = gr[i];
  const float mi = b1 * m[i] + omb1 * g;
  const float vi = b2 * v[i] + omb2 * g * g;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Z[r, :] = y[r, :] * (||P_r||^2)^(1 / (2 N)): the cores predicted for P~ = P / ||P|| scaled
// so that Psi of them approximates P itself (every core carries ||P||^(1/N)).
__global__ __launch_bounds__(256) void to_f64_kernel(const float* __restrict__ x, int64_t n,
                                                     int64_t per_row,
                                                     const double* __restrict__ pn2,
                                                     double inv2n, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = pn2 ? pow(pn2[i / per_row], inv2n) : 1.0;
  y[i] = (double)x[i] * sc;
}

// Row normalisation P~ = P / ||P|| (FP64 in, FP32 out), one work-group per row.
__global__ __launch_bounds__(256) void normalize_kernel(const double* __restrict__ P, int64_t d,
                                                        float* __restrict__ out) {
  __shared__ double red[16];
  const double* p = P + (int64_t)blockIdx.x * d;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) s += p[i] * p[i];
  s = block_sum(s, red);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  float* o = out + (int64_t)blockIdx.x * d;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) o[i] = (float)(p[i] * inv);
}

// Order-4 TR loss, one work-group per sample.  With A(i1, i2) = Z1(i1) Z2(i2) (R1 x R3) and
// C(i3, i4) = Z3(i3) Z4(i4) (R3 x R1), Psi = sum_{a, b} A[a, b] C[b, a]; D = Psi - target,
// loss = sum D^2, and gscale * d loss / d Z_n goes to dy (packed like y).
__global__ __launch_bounds__(256) void tr_loss4_kernel(const float* __restrict__ y,
                                                       const float* __restrict__ tgt, int dout,
                                                       TrLoss4 sh, float gscale,
                                                       float* __restrict__ loss,
                                                       float* __restrict__ dy) {
  extern __shared__ float lsm[];
  __shared__ double red[16];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int K1 = sh.K[0], K2 = sh.K[1], K3 = sh.K[2], K4 = sh.K[3];
  const int R1 = sh.R[0], R2 = sh.R[1], R3 = sh.R[2], R4 = sh.R[3];
  const int o1 = 0, o2 = o1 + R1 * K1 * R2, o3 = o2 + R2 * K2 * R3, o4 = o3 + R3 * K3 * R4;
  const int n12 = K1 * K2, n34 = K3 * K4, rr = R1 * R3;
  float* Z = lsm;                     // dout
  float* D = Z + sh.zpad;             // n12 x n34
  float* A = D + n12 * n34;           // n12 x (R1 R3), [a][b]
  float* C = A + n12 * rr;            // n34 x (R3 R1), [b][a]
  float* dA = C + n34 * rr;
  float* dC = dA + n12 * rr;
  const float* ys = y + (int64_t)s * dout;
  for (int e = tid; e < dout; e += 256) Z[e] = ys[e];
  __syncthreads();
  for (int e = tid; e < n12 * rr; e += 256) {
    const int i12 = e / rr, ab = e - i12 * rr, a = ab / R3, b = ab - a * R3;
    const int i1 = i12 / K2, i2 = i12 - i1 * K2;
    float acc = 0.f;
    for (int c = 0; c < R2; ++c)
      acc += Z[o1 + (a * K1 + i1) * R2 + c] * Z[o2 + (c * K2 + i2) * R3 + b];
    A[e] = acc;
  }
  for (int e = tid; e < n34 * rr; e += 256) {
    const int i34 = e / rr, ba = e - i34 * rr, b = ba / R1, a = ba - b * R1;
    const int i3 = i34 / K4, i4 = i34 - i3 * K4;
    float acc = 0.f;
    for (int d = 0; d < R4; ++d)
      acc += Z[o3 + (b * K3 + i3) * R4 + d] * Z[o4 + (d * K4 + i4) * R1 + a];
    C[e] = acc;
  }
  __syncthreads();
  const float* ts = tgt + (int64_t)s * n12 * n34;
  double part = 0.0;
  for (int e = tid; e < n12 * n34; e += 256) {
    const int i12 = e / n34, i34 = e - i12 * n34;
    const float* ar = A + i12 * rr;
    const float* cr = C + i34 * rr;
    float psi = 0.f;
    for (int a = 0; a < R1; ++a)
      for (int b = 0; b < R3; ++b) psi += ar[a * R3 + b] * cr[b * R1 + a];
    const float dv = psi - ts[e];
    D[e] = dv;
    part += (double)dv * dv;
  }
  const double l2 = block_sum(part, red);
  if (tid == 0) loss[s] = (float)l2;
  __syncthreads();
  const float g2 = 2.f * gscale;
  for (int e = tid; e < n12 * rr; e += 256) {
    const int i12 = e / rr, ab = e - i12 * rr, a = ab / R3, b = ab - a * R3;
    const float* drow = D + i12 * n34;
    float acc = 0.f;
    for (int i34 = 0; i34 < n34; ++i34) acc += drow[i34] * C[i34 * rr + b * R1 + a];
    dA[e] = g2 * acc;
  }
  for (int e = tid; e < n34 * rr; e += 256) {
    const int i34 = e / rr, ba = e - i34 * rr, b = ba / R1, a = ba - b * R1;
    float acc = 0.f;
    for (int i12 = 0; i12 < n12; ++i12) acc += D[i12 * n34 + i34] * A[i12 * rr + a * R3 + b];
    dC[e] = g2 * acc;
  }
  __syncthreads();
  float* dys = dy + (int64_t)s * dout;
  // dZ1[a, i1, c] = sum_{i2, b} dA(i1, i2)[a, b] Z2[c, i2, b]
  for (int e = tid; e < R1 * K1 * R2; e += 256) {
    const int a = e / (K1 * R2), r = e - a * K1 * R2, i1 = r / R2, c = r - i1 * R2;
    float acc = 0.f;
    for (int i2 = 0; i2 < K2; ++i2)
      for (int b = 0; b < R3; ++b)
        acc += dA[(i1 * K2 + i2) * rr + a * R3 + b] * Z[o2 + (c * K2 + i2) * R3 + b];
    dys[o1 + e] = acc;
  }
  // dZ2[c, i2, b] = sum_{i1, a} Z1[a, i1, c] dA(i1, i2)[a, b]
  for (int e = tid; e < R2 * K2 * R3; e += 256) {
    const int c = e / (K2 * R3), r = e - c * K2 * R3, i2 = r / R3, b = r - i2 * R3;
    float acc = 0.f;
    for (int i1 = 0; i1 < K1; ++i1)
      for (int a = 0; a < R1; ++a)
        acc += Z[o1 + (a * K1 + i1) * R2 + c] * dA[(i1 * K2 + i2) * rr + a * R3 + b];
    dys[o2 + e] = acc;
  }
  // dZ3[b, i3, d] = sum_{i4, a} dC(i3, i4)[b, a] Z4[d, i4, a]
  for (int e = tid; e < R3 * K3 * R4; e += 256) {
    const int b = e / (K3 * R4), r = e - b * K3 * R4, i3 = r / R4, d = r - i3 * R4;
    float acc = 0.f;
    for (int i4 = 0; i4 < K4; ++i4)
      for (int a = 0; a < R1; ++a)
        acc += dC[(i3 * K4 + i4) * rr + b * R1 + a] * Z[o4 + (d * K4 + i4) * R1 + a];
    dys[o3 + e] = acc;
  }
  // dZ4[d, i4, a] = sum_{i3, b} Z3[b, i3, d] dC(i3, i4)[b, a]
  for (int e = tid; e < R4 * K4 * R1; e += 256) {
    const int d = e / (K4 * R1), r = e - d * K4 * R1, i4 = r / R1, a = r - i4 * R1;
    float acc = 0.f;
    for (int i3 = 0; i3 < K3; ++i3)
      for (int b = 0; b < R3; ++b)
        acc += Z[o3 + (b * K3 + i3) * R4 + d] * dC[(i3 * K4 + i4) * rr + b * R1 + a];
    dys[o4 + e] = acc;
  }
}

// ---------------------------------------------------------------------------------------
hipError_t launch_gemm(bool bf, GemmArgs g, int slices, hipStream_t s) {
  const dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM),
                  (unsigned)slices);
  prof_begin("mlp_gemm", s);
  if (bf)
    hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(256), 0, s, g);
  prof_end(s);
  return hipGetLastError();
}

int gemm_slices(int64_t M, int64_t N, int64_t K, int64_t* kslice) {
  const int64_t tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  int64_t sl = (512 + tiles - 1) / tiles;
  const int64_t ksteps = (K + kBK - 1) / kBK;
  if (sl > ksteps) sl = ksteps;
  if (sl < 1) sl = 1;
  if (sl > 32) sl = 32;
  const int64_t per = ((ksteps + sl - 1) / sl) * kBK;
  *kslice = per;
  return (int)((K + per - 1) / per);
}

hipError_t launch_epilogue(const float* part, int slices, int64_t M, int64_t N,
                           const float* bias, const float* mask, int mode, float* out,
                           hipStream_t s) {
  const int64_t n = M * N;
  hipLaunchKernelGGL(epilogue_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                     slices, M, N, bias, mask, mode, out);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int64_t M, int64_t N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, G, M, N,
                     out);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, double lr,
                       double b1, double b2, double eps, int t, hipStream_t s) {
  // 1 - beta and the bias corrections from the double betas (1 - (float)0.999 alone is off
  // by 1e-5 relative)
  const float omb1 = (float)(1.0 - b1), omb2 = (float)(1.0 - b2);
  const float c1 = (float)(1.0 - pow(b1, t)), c2 = (float)(1.0 - pow(b2, t));
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, g, m, v,
                     n, (float)lr, (float)b1, (float)b2, omb1, omb2, (float)eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_f64(const float* x, int64_t n, int64_t per_row, const double* pn2, int order,
                         double* y, hipStream_t s) {
  hipLaunchKernelGGL(to_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     per_row, pn2, 1.0 / (2.0 * order), y);
  return hipGetLastError();
}

hipError_t launch_normalize(const double* P, int64_t d, int rows, float* out, hipStream_t s) {
  hipLaunchKernelGGL(normalize_kernel, dim3((unsigned)rows), dim3(256), 0, s, P, d, out);
  return hipGetLastError();
}

// Supervised core loss per sample: loss[s] = ||y[s] - t[s]||^2, dy[s] = gscale * 2 (y[s] - t[s]).
// One work-group per sample; the squares are summed per thread, then over the work-group in a
// fixed order.
__global__ __launch_bounds__(256) void core_loss_kernel(const float* __restrict__ y,
                                                        const float* __restrict__ t, int dout,
                                                        float gscale, float* __restrict__ loss,
                                                        float* __restrict__ dy) {
  __shared__ double red[16];
  const int64_t base = (int64_t)blockIdx.x * dout;
  double acc = 0.0;
  for (int i = threadIdx.x; i < dout; i += blockDim.x) {
    const float d = y[base + i] - t[base + i];
    acc += (double)d * d;
    dy[base + i] = gscale * 2.f * d;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) loss[blockIdx.x] = (float)acc;
}

hipError_t launch_core_loss(const float* y, const float* t, int dout, float gscale, int batch,
                            float* loss, float* dy, hipStream_t s) {
  prof_begin("mlp_core_loss", s);
  hipLaunchKernelGGL(core_loss_kernel, dim3((unsigned)batch), dim3(256), 0, s, y, t, dout, gscale,
                     loss, dy);
  prof_end(s);
  return hipGetLastError();
}

size_t tr_loss4_lds(const TrLoss4& sh) {
  const int n12 = sh.K[0] * sh.K[1], n34 = sh.K[2] * sh.K[3], rr = sh.R[0] * sh.R[2];
  return (size_t)(sh.zpad + n12 * n34 + 2 * (n12 + n34) * rr) * sizeof(float);
}

hipError_t launch_tr_loss4(const float* y, const float* tgt, int dout, const TrLoss4& sh,
                           float gscale, int batch, float* loss, float* dy, hipStream_t s) {
  const size_t lds = tr_loss4_lds(sh);
  hipError_t e = hipFuncSetAttribute((const void*)tr_loss4_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("mlp_tr_loss", s);
  hipLaunchKernelGGL(tr_loss4_kernel, dim3((unsigned)batch), dim3(256), lds, s, y, tgt, dout, sh,
                     gscale, loss, dy);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
