// Alg. 1 steps 4-5 for every mode in one read of X, with the Khatri-Rao structured test
// matrices (the structured-projection option named after Alg. 1), BF16 path; also ||X||^2.
//
// With X viewed as A contiguous slabs S_a of Ip x Iq (the last two modes sp = N-1, sq = N; slab
// a fixes the indices i_1 .. i_{N-2} of the other, "slab-index", modes) and the test matrix of
// mode n given by its Gaussian factors F^(n)_m (I_m x K_n), M_n[j, k] = prod_{m != n}
// F^(n)_m[i_m, k], every mode's sketch contribution from one slab is a product of the slab with
// one factor plus scalars of the slab's indices:
//   Y_sp[p, k] += c_sp(a, k) (S_a F^(sp)_sq)[p, k]
//   Y_sq[q, k] += c_sq(a, k) (S_a^T F^(sq)_sp)[q, k]
//   Y_n[i_n(a), k] += c_n(a, k) sum_p F^(n)_sp[p, k] (S_a F^(n)_sq)[p, k]   (n a slab-index mode)
// with c_n(a, k) the product of F^(n)_m[i_m(a), k] over the slab-index modes m != n.  So all N
// sketches come from one pass and only the factors (sum_m I_m K_n normals per mode) are drawn.
//
// Structure as the slab passes: one work-group streams whole slabs (the next slab's 16-byte
// loads in flight while the current one is processed), the slab in LDS as bf16; wave w owns
// row strip w and column strip w.  The products run on v_mfma_f32_16x16x32_bf16 against the
// factors, held in LDS as bf16 [k][i] for the whole launch.  Y_sp and Y_sq accumulate in the
// waves' registers; the column sums of the slab-index modes are reduced over the lane groups
// and the waves (per-wave values double-buffered by slab parity, summed in wave order after the
// next barrier) and added by one thread per (mode, k) to this work-group's partial of that mode
// in global memory.  Partials are summed in a fixed order by reduce_partials.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

namespace {

constexpr int kKaMaxI = 256;  // Ip, Iq bound
constexpr int kKaMaxK = 32;   // K_n bound (two 16-wide output tiles)

typedef unsigned short u16;

struct KaArgs {
  const float* X;
  int64_t A;
  int nidx;            // slab-index modes 0 .. nidx-1 (0-based), sp = nidx, sq = nidx + 1
  int Ip, Iq, nsp, nsq, ldS, ldQ, ldP, nwv;
  int dim[8];          // I_m
  int K[8];            // K'_m; 0 for a slab-index mode that is not projected
  int brow[8];         // first [k] row of mode n's operand in the row-strip buffer (n <= sp)
  int bq_rows;         // rows of the row-strip buffer
  const float* F;      // the factors
  int64_t foff[8][8];  // element offset of F^(n)_m (I_m x K_n row-major), m != n
  float* part[8];      // [grid][I_n][K_n] per projected mode
  double* xpart;       // [grid] partial sums of squares of X
};

__device__ __forceinline__ u16 bits16(float v) {
  const __bf16 b = (__bf16)v;
  return *(const u16*)&b;
}
__device__ __forceinline__ bf16x8 frag8(const u16* p) { return *(const bf16x8*)p; }
__device__ __forceinline__ bf16x8 frag8_col(const u16* p, int ld) {
  union {
    u16 h[8];
    bf16x8 v;
  } u;
#pragma unroll
  for (int j = 0; j < 8; ++j) u.h[j] = p[j * ld];
  return u.v;
}

// LDS: slab [Ip rounded up to 32][ldS] bf16 (the column-strip fragments read 32-row chunks;
// rows from Ip on stay zero), row-strip operands [bq_rows][ldQ] bf16, column-strip operand
// [K_sq][ldP] bf16, per-wave column sums [2][nwv][nidx][32] FP32, [nwv] FP64 for ||X||^2.
struct KaLayout {
  int oS, oBq, oBp, oD, oR, bytes;
  __host__ __device__ KaLayout(const KaArgs& p) {
    oS = 0;
    oBq = oS + (p.Ip + 31) / 32 * 32 * p.ldS * 2;
    oBp = oBq + p.bq_rows * p.ldQ * 2;
    oD = (oBp + p.K[p.nidx + 1] * p.ldP * 2 + 15) / 16 * 16;
    oR = oD + 2 * p.nwv * (p.nidx > 0 ? p.nidx : 1) * 32 * 4;
    bytes = oR + p.nwv * 8;
  }
};

// Slab a's indices of the slab-index modes (row-major, the first varies slowest).
__device__ __forceinline__ void slab_index(const KaArgs& p, int64_t a, int* idx) {
#pragma unroll
  for (int m = 7; m >= 0; --m)
    if (m < p.nidx) {
      idx[m] = (int)(a % p.dim[m]);
      a /= p.dim[m];
    }
}

// c_n(a, k): product of F^(n)_m[i_m, k] over the slab-index modes m != n.
__device__ __forceinline__ float slab_scale(const KaArgs& p, int n, const int* idx, int k) {
  float c = 1.f;
#pragma unroll
  for (int m = 0; m < 8; ++m)
    if (m < p.nidx && m != n) c *= p.F[p.foff[n][m] + (int64_t)idx[m] * p.K[n] + k];
  return c;
}

}  // namespace

template <int LDN>
__global__ __launch_bounds__(1024) void kr_allmode_kernel(KaArgs p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const KaLayout L(p);
  u16* Ss = (u16*)(smem_raw + L.oS);
  u16* Bq = (u16*)(smem_raw + L.oBq);
  u16* Bp = (u16*)(smem_raw + L.oBp);
  float* dpart = (float*)(smem_raw + L.oD);
  double* red = (double*)(smem_raw + L.oR);
  const int nth = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m16 = lane & 15, g4 = lane >> 4;
  const int Ip = p.Ip, Iq = p.Iq, ldS = p.ldS, ldQ = p.ldQ, ldP = p.ldP;
  const int sp = p.nidx, sq = p.nidx + 1;
  const int Kp = p.K[sp], Kq = p.K[sq];
  const int ncq = (Iq + 31) / 32, ncp = (Ip + 31) / 32;
  const int KpT = (Kp + 15) / 16, KqT = (Kq + 15) / 16;
  const bool rowW = wid < p.nsp, colW = wid < p.nsq;
  const int dstride = p.nwv * (p.nidx > 0 ? p.nidx : 1) * 32;  // one parity of dpart

  for (int x = tid; x < L.bytes / 4; x += nth) ((float*)smem_raw)[x] = 0.f;
  __syncthreads();
  // factors as bf16 operands: F^(n)_sq^T [k][i_q] for n <= sp, F^(sq)_sp^T [k][i_p]
  for (int n = 0; n <= sp; ++n) {
    const int K = p.K[n];
    const float* f = p.F + p.foff[n][sq];
    for (int x = tid; x < Iq * K; x += nth) {
      const int i = x / K, k = x % K;
      Bq[(p.brow[n] + k) * ldQ + i] = bits16(f[x]);
    }
  }
  {
    const float* f = p.F + p.foff[sq][sp];
    for (int x = tid; x < Ip * Kq; x += nth) {
      const int i = x / Kq, k = x % Kq;
      Bp[k * ldP + i] = bits16(f[x]);
    }
  }
  // this work-group's partials of the slab-index modes start at zero
  for (int n = 0; n < p.nidx; ++n)
    if (p.K[n] > 0) {
      const int64_t cnt = (int64_t)p.dim[n] * p.K[n];
      float* dst = p.part[n] + (int64_t)blockIdx.x * cnt;
      for (int64_t x = tid; x < cnt; x += nth) dst[x] = 0.f;
    }

  f32x4 accp[2], accq[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) accp[t] = accq[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  double xs = 0.0;  // this thread's share of ||X||^2

  const int n4 = Ip * Iq / 4;
  float4 buf[LDN];
  auto load = [&](int64_t a) {
    const float4* src = (const float4*)(p.X + a * (int64_t)Ip * Iq);
#pragma unroll
    for (int s = 0; s < LDN; ++s) {
      const int f = tid + nth * s;
      buf[s] = f < n4 ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // sum of the per-wave column sums of slab aa (parity par) into the slab-index partials
  auto fold = [&](int64_t aa, int par) {
    for (int x = tid; x < 32 * p.nidx; x += nth) {
      const int n = x >> 5, k = x & 31;
      if (k < p.K[n]) {
        int idx[8];
        slab_index(p, aa, idx);
        float d = 0.f;
        for (int w = 0; w < p.nsp; ++w) d += dpart[par * dstride + (w * p.nidx + n) * 32 + k];
        float* dst = p.part[n] + ((int64_t)blockIdx.x * p.dim[n] + idx[n]) * p.K[n] + k;
        *dst += slab_scale(p, n, idx, k) * d;
      }
    }
  };
  const int st_i0 = (4 * tid) / Iq, st_c0 = 4 * tid - st_i0 * Iq;
  const int st_di = (4 * nth) / Iq, st_dc = 4 * nth - st_di * Iq;

  int64_t a = blockIdx.x, aprev = -1;
  int lastpar = 0;
  if (a < p.A) load(a);
  for (int it = 0; a < p.A; a += gridDim.x, ++it) {
    __syncthreads();  // the previous slab's LDS reads and column sums are done
    if (aprev >= 0) fold(aprev, (it - 1) & 1);
    {
      int i = st_i0, c = st_c0;
      float sq = 0.f;
#pragma unroll
      for (int s = 0; s < LDN; ++s) {
        const int f = tid + nth * s;
        if (f < n4) {
          const float4 v = buf[s];
          sq += v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
          const uint32_t lo = (uint32_t)bits16(v.x) | ((uint32_t)bits16(v.y) << 16);
          const uint32_t hi = (uint32_t)bits16(v.z) | ((uint32_t)bits16(v.w) << 16);
          *(uint2*)(Ss + i * ldS + c) = make_uint2(lo, hi);
        }
        i += st_di;
        c += st_dc;
        if (c >= Iq) {
          c -= Iq;
          ++i;
        }
      }
      xs += (double)sq;
    }
    if (a + gridDim.x < p.A) load(a + gridDim.x);
    __syncthreads();
    int idx[8];
    slab_index(p, a, idx);
    const int par = it & 1;
    if (rowW) {
      const u16* arow = Ss + (16 * wid + m16) * ldS + 8 * g4;
      for (int n = 0; n <= sp; ++n) {
        const int K = p.K[n];
        if (K == 0) continue;
        const int KT = (K + 15) / 16;
        const u16* B = Bq + p.brow[n] * ldQ;
        f32x4 u[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        for (int c = 0; c < ncq; ++c) {
          const bf16x8 av = frag8(arow + 32 * c);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KT) u[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            av, frag8(B + min(16 * t + m16, K - 1) * ldQ + 32 * c + 8 * g4), u[t], 0, 0, 0);
        }
        // lane holds u[t][r] = (S F)[16 wid + 4 g4 + r][16 t + m16]
        if (n == sp) {
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KT) {
              const int k = min(16 * t + m16, K - 1);
              const float c = slab_scale(p, n, idx, k);
#pragma unroll
              for (int r = 0; r < 4; ++r) accp[t][r] += c * u[t][r];
            }
        } else {
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KT) {
              const int k = min(16 * t + m16, K - 1);
              const float* fl = p.F + p.foff[n][sp] + k;
              float d = 0.f;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 16 * wid + 4 * g4 + r;
                if (row < Ip) d += fl[(int64_t)row * K] * u[t][r];
              }
              d += __shfl_xor(d, 16);
              d += __shfl_xor(d, 32);
              if (g4 == 0 && 16 * t + m16 < K) dpart[par * dstride + (wid * p.nidx + n) * 32 + 16 * t + m16] = d;
            }
        }
      }
    }
    if (colW) {
      f32x4 v[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
      const u16* acol = Ss + (8 * g4) * ldS + 16 * wid + m16;
      for (int c = 0; c < ncp; ++c) {
        const bf16x8 av = frag8_col(acol + 32 * c * ldS, ldS);
#pragma unroll
        for (int t = 0; t < 2; ++t)
          if (t < KqT) v[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                          av, frag8(Bp + min(16 * t + m16, Kq - 1) * ldP + 32 * c + 8 * g4), v[t], 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
        if (t < KqT) {
          const float c = slab_scale(p, sq, idx, min(16 * t + m16, Kq - 1));
#pragma unroll
          for (int r = 0; r < 4; ++r) accq[t][r] += c * v[t][r];
        }
    }
    aprev = a;
    lastpar = par;
  }
  __syncthreads();
  if (aprev >= 0) fold(aprev, lastpar);
  // partials of the two slab modes: rows 16 wid + 4 g4 + r, columns 16 t + m16
  if (rowW) {
    float* dst = p.part[sp] + (int64_t)blockIdx.x * Ip * Kp;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * wid + 4 * g4 + r, k = 16 * t + m16;
        if (t < KpT && i < Ip && k < Kp) dst[i * Kp + k] = accp[t][r];
      }
  }
  if (colW) {
    float* dst = p.part[sq] + (int64_t)blockIdx.x * Iq * Kq;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * wid + 4 * g4 + r, k = 16 * t + m16;
        if (t < KqT && i < Iq && k < Kq) dst[i * Kq + k] = accq[t][r];
      }
  }
  // ||X||^2: wave sums, then the waves in order
  for (int o = 32; o > 0; o >>= 1) xs += __shfl_xor(xs, o);
  if (lane == 0) red[wid] = xs;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < p.nwv; ++w) s += red[w];
    p.xpart[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------------------
namespace {

bool ka_fill(KaArgs& p, int order, const int64_t* dims, const int* Keff) {
  if (order < 3 || order > 8) return false;
  p.nidx = order - 2;
  const int sp = p.nidx, sq = sp + 1;
  p.A = 1;
  for (int m = 0; m < sp; ++m) p.A *= dims[m];
  p.Ip = (int)dims[sp];
  p.Iq = (int)dims[sq];
  p.nsp = (p.Ip + 15) / 16;
  p.nsq = (p.Iq + 15) / 16;
  p.nwv = p.nsp > p.nsq ? p.nsp : p.nsq;
  p.ldS = (p.Iq + 31) / 32 * 32 + 8;
  p.ldQ = p.ldS;
  p.ldP = (p.Ip + 31) / 32 * 32 + 8;
  int rows = 0;
  for (int m = 0; m < order; ++m) {
    p.dim[m] = (int)dims[m];
    p.K[m] = Keff[m] < dims[m] ? Keff[m] : 0;  // not projected: no sketch
  }
  for (int n = 0; n <= sp; ++n) {
    p.brow[n] = rows;
    rows += p.K[n];
  }
  p.bq_rows = rows;
  return true;
}

}  // namespace

bool kr_allmode_supported(int order, const int64_t* dims, const int* Keff, const void* X) {
  KaArgs p{};
  if (!ka_fill(p, order, dims, Keff)) return false;
  const int sp = p.nidx, sq = sp + 1;
  if (p.Ip < 16 || p.Iq < 16 || p.Ip > kKaMaxI || p.Iq > kKaMaxI || p.Iq % 4 != 0) return false;
  if (p.K[sp] == 0 || p.K[sq] == 0) return false;  // both slab modes projected
  for (int m = 0; m < order; ++m)
    if (p.K[m] > kKaMaxK) return false;
  if (((uintptr_t)X & 15) != 0 || p.A < 256) return false;
  if ((int64_t)p.Ip * p.Iq / 4 > 16LL * 64 * p.nwv) return false;  // register staging
  return KaLayout(p).bytes <= 150 * 1024;
}

int64_t kr_allmode_grid(int order, const int64_t* dims) {
  int64_t A = 1;
  for (int m = 0; m < order - 2; ++m) A *= dims[m];
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipGetLastError();
  return A < cus ? A : cus;
}

hipError_t launch_kr_allmode(const void* X, int order, const int64_t* dims, const int* Keff,
                             const float* F, const int64_t (*foff)[8], float* const* part,
                             double* xpart, int64_t grid, hipStream_t s) {
  KaArgs p{};
  if (!ka_fill(p, order, dims, Keff)) return hipErrorInvalidValue;
  p.X = (const float*)X;
  p.F = F;
  for (int n = 0; n < order; ++n) {
    for (int m = 0; m < order; ++m) p.foff[n][m] = foff[n][m];
    p.part[n] = part[n];
  }
  p.xpart = xpart;
  const int nth = 64 * p.nwv;
  const bool l13 = (int64_t)p.Ip * p.Iq / 4 <= 13LL * nth;
  const void* fn = l13 ? (const void*)kr_allmode_kernel<13> : (const void*)kr_allmode_kernel<16>;
  const size_t lds = (size_t)KaLayout(p).bytes;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("sketch_kr_allmode", s);
  void* args[] = {&p};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(nth), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
