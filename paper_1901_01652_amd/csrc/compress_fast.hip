// Alg. 1 step 7 / Eq. (3), first stage: the products over the last two modes in one read of
// X.  With X viewed as A slabs of I1 x I2 (I1 = I_{N-1}, I2 = I_N, each slab contiguous),
//   T[a] = Q1^T X_a Q2        (K1 x K2 per slab, written in FP64)
// computed one block of 32 rows of the slab at a time:
//   S = X_blk Q2              (32 x K2, contraction over the slab's columns)
//   T[a] += Q1[blk]^T S       (K1 x K2, contraction over the block's rows)
// on the matrix cores.  The remaining modes are then contracted on the small T.
//
// BF16 path with FP32 refinement: X = X_hi + X_lo, Q = Q_hi + Q_lo, S = S_hi + S_lo split
// into bf16 pairs; every product takes hi*hi + hi*lo + lo*hi with FP32 accumulation, which
// keeps FP32-class accuracy while the data still stream as FP32 once.
// FP32 path: v_mfma_f32_16x16x4_f32 on FP32 operands.
//
// Work-groups are persistent over slabs; the next row block's 16-byte loads are in flight
// while the matrix cores work on the current one.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

constexpr int kCsTR = 32;        // smallest rows-per-item block (see cs_tr)
constexpr int kCsThreads = 512;  // 8 wavefronts
constexpr int kCsMaxI2 = 512;
constexpr int kCsMaxK = 64;

struct CsArgs {
  const float* X;
  int64_t A;
  int I1, I2, K1, K2;
  const double* Q1;  // I1 x K1 row-major
  const double* Q2;  // I2 x K2 row-major
  double* T;         // A x K1 x K2
  int ldX, kI2, ldS, vec4;
};

template <bool BF, int TR>
struct CsLayout {
  using T = typename Mma<BF>::T;
  int oXh, oXl, oQ2h, oQ2l, oQ1h, oQ1l, oSh, oSl, total;
  __host__ __device__ CsLayout(int K1, int K2, int ldX, int ldS) {
    const int a = 16 / (int)sizeof(T);
    auto up = [a](int v) { return (v + a - 1) / a * a; };
    const int K1p = (K1 + 15) / 16 * 16, K2p = (K2 + 15) / 16 * 16;
    const int np = BF ? 2 : 1;  // hi and lo parts
    int o = 0;
    oXh = o; o = up(o + TR * ldX);
    oXl = o; o = up(o + (np - 1) * TR * ldX);
    oQ2h = o; o = up(o + K2p * ldX);
    oQ2l = o; o = up(o + (np - 1) * K2p * ldX);
    oQ1h = o; o = up(o + K1p * ldS);
    oQ1l = o; o = up(o + (np - 1) * K1p * ldS);
    oSh = o; o = up(o + K2p * ldS);
    oSl = o; o = up(o + (np - 1) * K2p * ldS);
    total = o;
  }
};

template <bool BF>
__device__ __forceinline__ void split(float v, typename Mma<BF>::T& hi, typename Mma<BF>::T& lo) {
  if constexpr (BF) {
    hi = (__bf16)v;
    lo = (__bf16)(v - (float)hi);
  } else {
    hi = v;
    lo = 0.f;
  }
}

template <bool BF>
__device__ __forceinline__ f32x4 mma3(const typename Mma<BF>::T* Ah, const typename Mma<BF>::T* Al,
                                      int lda, const typename Mma<BF>::T* Bh,
                                      const typename Mma<BF>::T* Bl, int ldb, int kdim, f32x4 acc) {
  acc = tile_abt(Ah, lda, Bh, ldb, kdim, acc);
  if constexpr (BF) {
    acc = tile_abt(Ah, lda, Bl, ldb, kdim, acc);
    acc = tile_abt(Al, lda, Bh, ldb, kdim, acc);
  }
  return acc;
}

// TR: rows of the slab per item (64 when TR * I2 fits the register staging, else 32).
template <bool BF, int TR>
__global__ __launch_bounds__(kCsThreads, 2) void compress_slab_kernel(CsArgs p) {
  using T = typename Mma<BF>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = (T*)smem_raw;
  const CsLayout<BF, TR> L(p.K1, p.K2, p.ldX, p.ldS);
  T* Xh = sm + L.oXh;
  T* Xl = sm + L.oXl;
  T* Q2h = sm + L.oQ2h;
  T* Q2l = sm + L.oQ2l;
  T* Q1h = sm + L.oQ1h;
  T* Q1l = sm + L.oQ1l;
  T* Sh = sm + L.oSh;
  T* Sl = sm + L.oSl;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int I1 = p.I1, I2 = p.I2, K1 = p.K1, K2 = p.K2, ldX = p.ldX, ldS = p.ldS;
  const int K1T = (K1 + 15) / 16, K2T = (K2 + 15) / 16;
  const int nblk = (I1 + TR - 1) / TR;

  for (int x = tid; x < L.total; x += kCsThreads) sm[x] = Mma<BF>::cvt(0.f);
  __syncthreads();
  for (int x = tid; x < I2 * K2; x += kCsThreads) {
    const int i = x / K2, k = x % K2;
    T hi, lo;
    split<BF>((float)p.Q2[x], hi, lo);
    Q2h[k * ldX + i] = hi;
    if (BF) Q2l[k * ldX + i] = lo;
  }

  const int64_t nitems = p.A * nblk;  // (slab, row block) pairs, slab-major
  float4 buf[8];
  auto load = [&](int64_t item) {
    const int64_t a = item / nblk;
    const int r0 = (int)(item % nblk) * TR;
    const int rows = min(TR, I1 - r0);
    const float* src = p.X + (a * I1 + r0) * (int64_t)I2;
    const int n = rows * I2;
    if (p.vec4) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int f = tid + kCsThreads * s;
        buf[s] = (4 * f < n) ? *(const float4*)(src + 4 * f) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int f = tid + kCsThreads * s;
        float4 v;
        v.x = (4 * f + 0 < n) ? src[4 * f + 0] : 0.f;
        v.y = (4 * f + 1 < n) ? src[4 * f + 1] : 0.f;
        v.z = (4 * f + 2 < n) ? src[4 * f + 2] : 0.f;
        v.w = (4 * f + 3 < n) ? src[4 * f + 3] : 0.f;
        buf[s] = v;
      }
    }
  };
  // (row, column) of the first of this thread's 4 elements in each of its 8 float4 slots,
  // fixed for every item: the stores below advance it with a carry instead of dividing
  int il_s[8], c_s[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int x0 = 4 * (tid + kCsThreads * s);
    il_s[s] = x0 / I2;
    c_s[s] = x0 - il_s[s] * I2;
  }
  auto store = [&](int64_t item) {
    const int r0 = (int)(item % nblk) * TR;
    const int rows = min(TR, I1 - r0);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float vv[4] = {buf[s].x, buf[s].y, buf[s].z, buf[s].w};
      int il = il_s[s], c = c_s[s];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (il < TR) {
          T hi, lo;
          split<BF>(il < rows ? vv[e] : 0.f, hi, lo);
          Xh[il * ldX + c] = hi;
          if (BF) Xl[il * ldX + c] = lo;
        }
        if (++c == I2) {
          c = 0;
          ++il;
        }
      }
    }
    for (int x = tid; x < TR * K1; x += kCsThreads) {
      const int il = x / K1, k = x % K1;
      T hi, lo;
      split<BF>(il < rows ? (float)p.Q1[(int64_t)(r0 + il) * K1 + k] : 0.f, hi, lo);
      Q1h[k * ldS + il] = hi;
      if (BF) Q1l[k * ldS + il] = lo;
    }
  };

  f32x4 tacc[2];
  tacc[0] = tacc[1] = f32x4{0.f, 0.f, 0.f, 0.f};
  // contiguous range of items per work-group, whole slabs only
  const int64_t per = (p.A + gridDim.x - 1) / gridDim.x;
  const int64_t a_begin = (int64_t)blockIdx.x * per;
  const int64_t a_end = min(p.A, a_begin + per);
  int64_t item = a_begin * nblk;
  const int64_t item_end = a_end * nblk;
  if (item < item_end) load(item);
  for (; item < item_end; ++item) {
    store(item);
    __syncthreads();
    if (item + 1 < item_end) load(item + 1);
    // S [TR x K2] = X_blk [TR x I2] * Q2 [I2 x K2]; tiles q = wid + 8 s, (mt, nt) = q / K2T
    for (int q = wid; q < (TR / 16) * K2T; q += 8) {
      const int mt = q / K2T, nt = q % K2T;
      f32x4 sacc = mma3<BF>(Xh + mt * 16 * ldX, Xl + mt * 16 * ldX, ldX, Q2h + nt * 16 * ldX,
                            Q2l + nt * 16 * ldX, ldX, p.kI2, f32x4{0.f, 0.f, 0.f, 0.f});
      const int col = nt * 16 + (lane & 15);  // k2
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = mt * 16 + 4 * (lane >> 4) + r;  // il
        T hi, lo;
        split<BF>(sacc[r], hi, lo);
        Sh[col * ldS + row] = hi;
        if (BF) Sl[col * ldS + row] = lo;
      }
    }
    __syncthreads();
    // T [K1 x K2] += Q1[blk]^T [K1 x 32] * S [32 x K2]; tiles q = wid + 8 s
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int q = wid + 8 * s;
      if (q < K1T * K2T) {
        const int mt = q / K2T, nt = q % K2T;
        tacc[s] = mma3<BF>(Q1h + mt * 16 * ldS, Q1l + mt * 16 * ldS, ldS, Sh + nt * 16 * ldS,
                           Sl + nt * 16 * ldS, ldS, TR, tacc[s]);
      }
    }
    if ((item + 1) % nblk == 0) {  // slab done: write T[a], reset
      const int64_t a = item / nblk;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int q = wid + 8 * s;
        if (q < K1T * K2T) {
          const int mt = q / K2T, nt = q % K2T;
          const int k2 = nt * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k1 = mt * 16 + 4 * (lane >> 4) + r;
            if (k1 < K1 && k2 < K2) p.T[(a * K1 + k1) * K2 + k2] = (double)tacc[s][r];
          }
        }
        tacc[s] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Rows per item: 64 when 64 x I2 fits the register staging (32 float4 per thread), else 32.
static int cs_tr(int64_t I2) { return 64 * I2 <= 4LL * 8 * kCsThreads ? 64 : 32; }

static void cs_dims(bool bf, int I2, int& ldX, int& kI2, int& ldS) {
  kI2 = bf ? (I2 + 31) / 32 * 32 : (I2 + 3) / 4 * 4;
  ldX = kI2 + (bf ? 8 : 2);
  ldS = cs_tr(I2) + (bf ? 8 : 2);
}

static size_t cs_lds(bool bf, int I2, int K1, int K2) {
  int ldX, kI2, ldS;
  cs_dims(bf, I2, ldX, kI2, ldS);
  const bool tr64 = cs_tr(I2) == 64;
  const int total = bf ? (tr64 ? CsLayout<true, 64>(K1, K2, ldX, ldS).total
                               : CsLayout<true, 32>(K1, K2, ldX, ldS).total)
                       : (tr64 ? CsLayout<false, 64>(K1, K2, ldX, ldS).total
                               : CsLayout<false, 32>(K1, K2, ldX, ldS).total);
  return (size_t)total * (bf ? 2 : 4);
}

bool compress_slab_supported(Arith ar, int64_t A, int64_t I1, int64_t I2, int K1, int K2) {
  if (ar == kF64) return false;
  if (I2 > kCsMaxI2 || K1 > kCsMaxK || K2 > kCsMaxK || I1 > (1 << 20)) return false;
  if ((int64_t)kCsTR * I2 > 4LL * 8 * kCsThreads) return false;  // register staging
  if (A < 256) return false;  // too few slabs to fill the device
  return cs_lds(ar == kBF16, (int)I2, K1, K2) <= 150 * 1024;
}

hipError_t launch_compress_slab(Arith ar, const void* X, int64_t A, int64_t I1, int64_t I2,
                                int K1, int K2, const double* Q1, const double* Q2, double* T,
                                hipStream_t s) {
  const bool bf = ar == kBF16;
  CsArgs p{};
  p.X = (const float*)X;
  p.A = A;
  p.I1 = (int)I1;
  p.I2 = (int)I2;
  p.K1 = K1;
  p.K2 = K2;
  p.Q1 = Q1;
  p.Q2 = Q2;
  p.T = T;
  cs_dims(bf, (int)I2, p.ldX, p.kI2, p.ldS);
  p.vec4 = (((uintptr_t)X & 15) == 0) && (I2 % 4 == 0);
  const size_t lds = cs_lds(bf, (int)I2, K1, K2);
  const bool tr64 = cs_tr(I2) == 64;
  const void* fn = bf ? (tr64 ? (const void*)compress_slab_kernel<true, 64>
                              : (const void*)compress_slab_kernel<true, 32>)
                      : (tr64 ? (const void*)compress_slab_kernel<false, 64>
                              : (const void*)compress_slab_kernel<false, 32>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kCsThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  (void)hipGetLastError();
  int64_t grid = (int64_t)cus * per_cu;
  if (grid > A) grid = A;
  prof_begin("compress_fused", s);
  void* args[] = {&p};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kCsThreads), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
