// Alg. 1 step 7 / Eq. (3), first stage, BF16 path with FP32 refinement: the products over the
// last two modes in one read of X, one wavefront per slab.  With X viewed as A contiguous slabs
// S_a of Ip x Iq (Ip = I_{N-1}, Iq = I_N):
//   T[a] = Q_{N-1}^T S_a Q_N      (Kp x Kq per slab, written in FP64)
// Each wavefront streams whole slabs on its own, 16 rows (one strip) at a time, with no
// work-group barrier: lane (m, g) loads row 16s + m, columns 32c + 8g .. 32c + 8g + 7 of strip s
// straight into the A operand of v_mfma_f32_16x16x32_bf16 (the next strip's loads are in flight
// while the current one is multiplied), and
//   U = S_strip Q_N       bf16 products hi*hi + hi*lo + lo*hi, S = S_hi + S_lo and
//                         Q_N = Q_hi + Q_lo split into bf16 pairs, FP32 accumulation
//   T += Q_{N-1}[strip]^T U   on the FP32 matrix cores (v_mfma_f32_16x16x4_f32): the
//                         accumulator layout of U (lane (n, g) holds rows 4g .. 4g+3 of column
//                         n) is the B operand of four steps whose contraction runs over those
//                         rows, so U never leaves the registers.
// The data stream as FP32 once; the refinement keeps P at FP32-class accuracy.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

namespace {

constexpr int kCwThreads = 256;  // 4 wavefronts per work-group, two work-groups per CU
constexpr int kCwMaxI = 256;     // Ip, Iq bound
constexpr int kCwMaxK = 32;      // Kp, Kq bound (two 16-wide tiles)

struct CwArgs {
  const float* X;
  int64_t A;
  int Ip, Iq, Kp, Kq;
  int ldQ;           // pitch of the bf16 Q_N^T buffers [k][i_q]
  const double* Qp;  // Ip x Kp row-major
  const double* Qq;  // Iq x Kq row-major
  double* T;         // A x Kp x Kq
};

typedef unsigned short u16;

__device__ __forceinline__ u16 bf16_of(float v) {
  const __bf16 b = (__bf16)v;
  return *(const u16*)&b;
}
__device__ __forceinline__ float f32_of(u16 h) { return __uint_as_float((uint32_t)h << 16); }

union Frag {
  u16 h[8];
  bf16x8 v;
};

}  // namespace

// NC: 32-wide column chunks per strip (ceil(Iq / 32)).
template <int NC>
__global__ __launch_bounds__(kCwThreads, 2) void compress_wave_kernel(CwArgs p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ldQ = p.ldQ, Ip = p.Ip, Iq = p.Iq, Kp = p.Kp, Kq = p.Kq;
  u16* Qh = (u16*)smem_raw;          // Q_N^T hi [Kq][ldQ]
  u16* Ql = Qh + Kq * ldQ;           // Q_N^T lo
  float* Qpf = (float*)(Ql + Kq * ldQ);  // Q_{N-1} [Ip padded to 16][32] FP32, zero beyond Kp
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m16 = lane & 15, g4 = lane >> 4;
  const int nsp = (Ip + 15) / 16;
  const int KpT = (Kp + 15) / 16, KqT = (Kq + 15) / 16;

  for (int x = tid; x < Kq * ldQ; x += kCwThreads) {
    const int k = x / ldQ, i = x % ldQ;
    float v = i < Iq ? (float)p.Qq[i * Kq + k] : 0.f;
    const u16 h = bf16_of(v);
    Qh[x] = h;
    Ql[x] = bf16_of(v - f32_of(h));
  }
  for (int x = tid; x < nsp * 16 * 32; x += kCwThreads) {
    const int i = x / 32, k = x % 32;
    Qpf[x] = (i < Ip && k < Kp) ? (float)p.Qp[i * Kp + k] : 0.f;
  }
  __syncthreads();

  const int64_t wave = (int64_t)blockIdx.x * (kCwThreads / 64) + wid;
  const int64_t nwaves = (int64_t)gridDim.x * (kCwThreads / 64);
  // a wave takes whole slabs a = wave, wave + nwaves, .., strip by strip
  float4 f[NC][2];
  auto load = [&](int64_t a, int s) {
    const int row = 16 * s + m16;
    const float* src = p.X + (a * Ip + row) * (int64_t)Iq + 8 * g4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int col = 32 * c + 8 * g4;  // Iq % 4 == 0: each float4 is in or out whole
      const bool ok0 = row < Ip && col < Iq, ok1 = row < Ip && col + 4 < Iq;
      f[c][0] = ok0 ? *(const float4*)(src + 32 * c) : make_float4(0.f, 0.f, 0.f, 0.f);
      f[c][1] = ok1 ? *(const float4*)(src + 32 * c + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  int64_t a = wave;
  int s = 0;
  if (a < p.A) load(a, 0);
  f32x4 tacc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) tacc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  while (a < p.A) {
    // split the strip into bf16 pairs
    Frag hi[NC], lo[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float v[8] = {f[c][0].x, f[c][0].y, f[c][0].z, f[c][0].w,
                          f[c][1].x, f[c][1].y, f[c][1].z, f[c][1].w};
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const u16 h = bf16_of(v[j]);
        hi[c].h[j] = h;
        lo[c].h[j] = bf16_of(v[j] - f32_of(h));
      }
    }
    // the next strip (or the next slab's first) in flight during the products
    const int row0 = 16 * s;
    int64_t na = a;
    int ns = s + 1;
    if (ns == nsp) {
      ns = 0;
      na = a + nwaves;
    }
    if (na < p.A) load(na, ns);
    // U [16 x Kq] = S_strip Q_N (three bf16 products)
    f32x4 u[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (t < KqT) {
          const int kr = min(16 * t + m16, Kq - 1);  // rows k >= Kq only feed discarded columns
          const bf16x8 qh = *(const bf16x8*)(Qh + kr * ldQ + 32 * c + 8 * g4);
          const bf16x8 ql = *(const bf16x8*)(Ql + kr * ldQ + 32 * c + 8 * g4);
          u[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[c].v, qh, u[t], 0, 0, 0);
          u[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[c].v, ql, u[t], 0, 0, 0);
          u[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[c].v, qh, u[t], 0, 0, 0);
        }
      }
    }
    // T [Kp x Kq] += Q_{N-1}[strip]^T U: step r contracts over rows 4 g + r of the strip;
    // lane (n = k_q, g) supplies U[4g + r][n] = u[t][r], lane (m = k_p, g) Q_{N-1}[row][m]
#pragma unroll
    for (int tp = 0; tp < 2; ++tp) {
      if (tp < KpT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float qa = Qpf[(row0 + 4 * g4 + r) * 32 + 16 * tp + m16];
#pragma unroll
          for (int tq = 0; tq < 2; ++tq)
            if (tq < KqT)
              tacc[tp][tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa, u[tq][r], tacc[tp][tq], 0, 0, 0);
        }
      }
    }
    if (s == nsp - 1) {  // slab done: T[a] (row k_p = 16 tp + 4 g + r, column k_q = 16 tq + m)
      double* dst = p.T + a * (int64_t)Kp * Kq;
#pragma unroll
      for (int tp = 0; tp < 2; ++tp)
#pragma unroll
        for (int tq = 0; tq < 2; ++tq) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int kp = 16 * tp + 4 * g4 + r, kq = 16 * tq + m16;
            if (tp < KpT && tq < KqT && kp < Kp && kq < Kq) dst[kp * Kq + kq] = (double)tacc[tp][tq][r];
          }
          tacc[tp][tq] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    a = na;
    s = ns;
  }
}

// ---------------------------------------------------------------------------------------
namespace {
int cw_ldq(int64_t Iq) { return (int)((Iq + 31) / 32 * 32 + 8); }
size_t cw_lds(int64_t Ip, int64_t Iq, int Kq) {
  const int nsp = (int)((Ip + 15) / 16);
  return (size_t)2 * Kq * cw_ldq(Iq) * 2 + (size_t)nsp * 16 * 32 * 4;
}
}  // namespace

bool compress_wave_supported(int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq, const void* X) {
  if (Ip < 1 || Iq < 4 || Ip > kCwMaxI || Iq > kCwMaxI || Iq % 4 != 0) return false;
  if (Kp < 1 || Kq < 1 || Kp > kCwMaxK || Kq > kCwMaxK) return false;
  if (((uintptr_t)X & 15) != 0 || A < 512) return false;
  return cw_lds(Ip, Iq, Kq) <= 64 * 1024;
}

hipError_t launch_compress_wave(const void* X, int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq,
                                const double* Qp, const double* Qq, double* T, hipStream_t s) {
  CwArgs p{};
  p.X = (const float*)X;
  p.A = A;
  p.Ip = (int)Ip;
  p.Iq = (int)Iq;
  p.Kp = Kp;
  p.Kq = Kq;
  p.ldQ = cw_ldq(Iq);
  p.Qp = Qp;
  p.Qq = Qq;
  p.T = T;
  const int nc = (int)((Iq + 31) / 32);
  const void* fn = nc <= 2 ? (const void*)compress_wave_kernel<2>
                 : nc <= 4 ? (const void*)compress_wave_kernel<4>
                 : nc <= 7 ? (const void*)compress_wave_kernel<7>
                           : (const void*)compress_wave_kernel<8>;
  const size_t lds = cw_lds(Ip, Iq, Kq);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipGetLastError();
  int64_t grid = (int64_t)cus * 2;
  const int64_t need = (A + 3) / 4;  // four wavefronts per work-group, one slab each at least
  if (grid > need) grid = need;
  prof_begin("compress_fused", s);
  void* args[] = {&p};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kCwThreads), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
