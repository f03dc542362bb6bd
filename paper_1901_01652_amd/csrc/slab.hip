// Passes over X in contiguous slabs of its last two modes, for the BF16 path.  With X viewed as
// A slabs S_a of Ip x Iq (Ip = I_{N-1}, Iq = I_N; slab a = the rows with i_1..i_{N-2} fixed,
// contiguous in memory), both trailing modes are served by one read of X:
//
//   op 0, sketch (Alg. 1 steps 4-5) of modes N-1 and N:
//     Y_{N-1} += S_a Mp_a,   Mp_a = rows a*Iq .. a*Iq+Iq-1 of the Gaussian matrix of mode N-1
//     Y_N     += S_a^T Mq_a, Mq_a = rows a*Ip .. a*Ip+Ip-1 of the Gaussian matrix of mode N
//   (the rows of mode n's Gaussian matrix are the row-major multi-indices of the other modes,
//   so a slab's block is one contiguous run of the stream: drawn once per slab, the ideal count)
//
//   op 1, one round of subspace iteration (the power iteration named after Alg. 1) of both:
//     U = S_a Q_N,  V = S_a^T Q_{N-1},  Y'_{N-1} += S_a V,  Y'_N += S_a^T U
//   (the fibers of both modes are complete inside a slab, so X_(n) X_(n)^T Q_n needs no second
//   read of X).
//
// Each work-group streams whole slabs: every thread loads its share of the next slab with
// 16-byte loads while the current one is processed; the slab is stored in LDS as bf16 (round to
// nearest even), row-major.  Wave w owns row strip w (rows 16w..16w+15: products contracting
// over the columns, A fragments read as 16-byte rows) and column strip w (columns 16w..16w+15:
// products contracting over the rows, fragments read with transposing LDS loads).  Products are
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; each wave keeps its share of Y_{N-1} and
// Y_N in accumulators across all its slabs and writes one partial per work-group, summed in a
// fixed order by reduce_partials.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

namespace {

constexpr int kSbMaxI = 256;  // Ip, Iq bound: 16 strips of 16
constexpr int kSbMaxK = 32;   // Kp, Kq bound: two 16-wide output tiles
constexpr int kSbLoads = 16;  // most 16-byte loads per thread per slab (register staging)

struct SlabArgs {
  const float* X;
  int64_t A;
  int Ip, Iq, Kp, Kq;
  int nsp, nsq;      // strips of 16 rows / columns
  int ldS;           // LDS row pitch of the slab (bf16 elements)
  int ldP, ldQ;      // pitch of the [k][i_p] and [k][i_q] operand buffers
  uint64_t seed;
  uint32_t swp, swq, tid;
  const double* Qp;  // Ip x Kp row-major (power step)
  const double* Qq;  // Iq x Kq row-major
  float* partp;      // [grid][Ip][Kp]
  float* partq;      // [grid][Iq][Kq]
};

// Offsets (bf16 elements) of the LDS buffers.  The [k][i] operand buffers hold K rows: the
// second 16-row tile reads its rows k >= K at row K - 1 instead, which only feeds output
// columns k >= K, never written out.
//   sketch: A, B = Mp^T [k][i_q], Mq^T [k][i_p] of the even slab step; C, D = of the odd one
//   power:  A, B = Q_{N-1}^T [k][i_p], Q_N^T [k][i_q];  C, D = U^T [k_q][i_p], V^T [k_p][i_q]
struct SlabLayout {
  int oS, oA, oB, oC, oD, total;
  __host__ __device__ SlabLayout(const SlabArgs& p, int op) {
    const int KpP = p.Kp, KqP = p.Kq;
    oS = 0;
    oA = oS + p.nsp * 16 * p.ldS;
    oB = oA + (op == 0 ? KpP * p.ldQ : KpP * p.ldP);
    oC = oB + (op == 0 ? KqP * p.ldP : KqP * p.ldQ);
    oD = oC + (op == 0 ? KpP * p.ldQ : KqP * p.ldP);
    total = oD + (op == 0 ? KqP * p.ldP : KpP * p.ldQ);
  }
};

typedef unsigned short u16;

__device__ __forceinline__ u16 bf16_bits(float v) {
  const __bf16 b = (__bf16)v;
  return *(const u16*)&b;
}

__device__ __forceinline__ f32x4 mma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 8 contiguous bf16 (16-byte aligned).
__device__ __forceinline__ bf16x8 frag_row(const u16* p) { return *(const bf16x8*)p; }

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// Column fragment of a row-major LDS tile: lane 16 g + m gets the 8 values of column m at rows
// 8 g .. 8 g + 7, the MFMA operand layout, from two transposing reads (ds_read_b64_tr_b16).
// Each lane names one 8-byte run of a row: within a 16-lane block, output lane 4 q + e receives
// element e of the runs named by lanes q, q + 4, q + 8, q + 12 (in that order).  So lane
// 16 g + r names row 8 g + (r >> 2) (+ 4 for the second read), columns 4 (r & 3) .. + 3;
// ``p`` is that address for the first read (row pitch ld, a multiple of 4).
__device__ __forceinline__ bf16x8 frag_col_tr(const u16* p, int ld) {
  const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)p);
  const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + 4 * ld));
  union {
    s16x4 h[2];
    bf16x8 v;
  } u;
  u.h[0] = lo;
  u.h[1] = hi;
  return u.v;
}

// The Gaussian blocks of slab a: Mp = rows a*Iq .. of mode N-1's matrix (Iq x Kp) into
// dstP[k][i_q], Mq = rows a*Ip .. of mode N's (Ip x Kq) into dstQ[k][i_p].  Block element x =
// i*K + k is stream element a*rows*K + x.  Each thread's calls advance by a fixed stride, so
// the (i, k) of its first element is carried forward instead of divided out.
__device__ __forceinline__ void draw_blocks(const SlabArgs& p, int64_t a, u16* dstP, u16* dstQ) {
  const int nth = blockDim.x, tid = threadIdx.x;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int rows = blk ? p.Ip : p.Iq, K = blk ? p.Kq : p.Kp, ld = blk ? p.ldP : p.ldQ;
    u16* dst = blk ? dstQ : dstP;
    const uint32_t sw = blk ? p.swq : p.swp;
    const int span = rows * K;
    const uint64_t e0 = (uint64_t)a * (uint64_t)span;
    const uint64_t c0 = e0 >> 2;
    const int off = (int)(e0 - 4 * c0);
    const int ncalls = (off + span + 3) >> 2;
    // element x of call ci, lane l: x = 4 ci + l - off; start at ci = tid (x may be < 0)
    const int x = 4 * tid - off;
    int i = x >= 0 ? x / K : -((-x + K - 1) / K);  // floor(x / K); x >= -3
    int k = x - i * K;
    const int stride = 4 * nth, di = stride / K, dk = stride - di * K;
    for (int ci = tid; ci < ncalls; ci += nth) {
      float z[4];
      normals4(p.seed, sw, p.tid, c0 + ci, z);
      int ii = i, kk = k;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        if (ii >= 0 && ii < rows) dst[kk * ld + ii] = bf16_bits(z[l]);
        if (++kk == K) {
          kk = 0;
          ++ii;
        }
      }
      i += di;
      k += dk;
      if (k >= K) {
        k -= K;
        ++i;
      }
    }
  }
}

}  // namespace

// LDN: 16-byte loads per thread per slab (the staging registers of the next slab).
template <int OP, int LDN>
__global__ __launch_bounds__(1024) void slab_pass_kernel(SlabArgs p) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  u16* sm = (u16*)smem_raw;
  const SlabLayout L(p, OP);
  u16* Ss = sm + L.oS;
  u16* Ba = sm + L.oA;
  u16* Bb = sm + L.oB;
  u16* Bc = sm + L.oC;
  u16* Bd = sm + L.oD;
  const int nth = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m16 = lane & 15, g4 = lane >> 4;
  const int Ip = p.Ip, Iq = p.Iq, Kp = p.Kp, Kq = p.Kq, ldS = p.ldS, ldP = p.ldP, ldQ = p.ldQ;
  const int ncq = (Iq + 31) / 32, ncp = (Ip + 31) / 32;  // 32-wide contraction chunks
  const int KpT = (Kp + 15) / 16, KqT = (Kq + 15) / 16;
  const bool rowW = wid < p.nsp, colW = wid < p.nsq;

  for (int x = tid; x < L.total; x += nth) sm[x] = 0;
  __syncthreads();
  if (OP == 1) {  // Q_{N-1}^T [k][i_p] into Ba, Q_N^T [k][i_q] into Bb (bf16)
    for (int x = tid; x < Ip * Kp; x += nth) {
      const int i = x / Kp, k = x % Kp;
      Ba[k * ldP + i] = bf16_bits((float)p.Qp[x]);
    }
    for (int x = tid; x < Iq * Kq; x += nth) {
      const int i = x / Kq, k = x % Kq;
      Bb[k * ldQ + i] = bf16_bits((float)p.Qq[x]);
    }
  }

  f32x4 accp[2], accq[2];  // row strip: Y_{N-1} rows x k tiles; column strip: Y_N
#pragma unroll
  for (int t = 0; t < 2; ++t) accp[t] = accq[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int n4 = Ip * Iq / 4;  // float4 per slab (Iq % 4 == 0)
  float4 buf[LDN];
  auto load = [&](int64_t a) {
    const float4* src = (const float4*)(p.X + a * (int64_t)Ip * Iq);
#pragma unroll
    for (int s = 0; s < LDN; ++s) {
      const int f = tid + nth * s;
      buf[s] = f < n4 ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };

  // (row, column) of this thread's first element in the slab, and the advance per load step
  const int st_i0 = (4 * tid) / Iq, st_c0 = 4 * tid - st_i0 * Iq;
  const int st_di = (4 * nth) / Iq, st_dc = 4 * nth - st_di * Iq;

  int64_t a = blockIdx.x;
  if (a < p.A) {
    load(a);
    if (OP == 0) draw_blocks(p, a, Ba, Bb);
  }
  for (int it = 0; a < p.A; a += gridDim.x, ++it) {
    __syncthreads();  // the previous slab's LDS reads are done
    // the slab into LDS as bf16, row-major
    {
      // the walk is restarted from values the compiler must treat as new each slab: left
      // loop-invariant, the store addresses are hoisted and spill to scratch, read back every
      // slab
      int i = st_i0, c = st_c0;
      asm volatile("" : "+v"(i), "+v"(c));
#pragma unroll
      for (int s = 0; s < LDN; ++s) {
        const int f = tid + nth * s;
        if (f < n4) {
          const float4 v = buf[s];
          const uint32_t lo = (uint32_t)bf16_bits(v.x) | ((uint32_t)bf16_bits(v.y) << 16);
          const uint32_t hi = (uint32_t)bf16_bits(v.z) | ((uint32_t)bf16_bits(v.w) << 16);
          *(uint2*)(Ss + i * ldS + c) = make_uint2(lo, hi);
        }
        i += st_di;
        c += st_dc;
        if (c >= Iq) {
          c -= Iq;
          ++i;
        }
      }
    }
    if (a + gridDim.x < p.A) load(a + gridDim.x);  // in flight while this slab is processed
    __syncthreads();
    // sketch: this slab's Gaussian blocks were drawn into the buffers of its parity
    u16* Mp = (it & 1) ? Bc : Ba;
    u16* Mq = (it & 1) ? Bd : Bb;
    if (OP == 0) {
      if (rowW) {  // Y_{N-1}[strip rows] += S Mp   (contraction over i_q)
        const u16* arow = Ss + (16 * wid + m16) * ldS + 8 * g4;
        for (int c = 0; c < ncq; ++c) {
          const bf16x8 av = frag_row(arow + 32 * c);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KpT) accp[t] = mma16(av, frag_row(Mp + min(16 * t + m16, Kp - 1) * ldQ + 32 * c + 8 * g4), accp[t]);
        }
      }
      if (colW) {  // Y_N[strip cols] += S^T Mq   (contraction over i_p)
        const u16* acol = Ss + (8 * g4 + (m16 >> 2)) * ldS + 16 * wid + 4 * (m16 & 3);
        for (int c = 0; c < ncp; ++c) {
          const bf16x8 av = frag_col_tr(acol + 32 * c * ldS, ldS);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KqT) accq[t] = mma16(av, frag_row(Mq + min(16 * t + m16, Kq - 1) * ldP + 32 * c + 8 * g4), accq[t]);
        }
      }
      // the next slab's Gaussian blocks into the other parity's buffers (no wave reads them
      // until after the next barrier)
      if (a + gridDim.x < p.A) draw_blocks(p, a + gridDim.x, (it & 1) ? Ba : Bc, (it & 1) ? Bb : Bd);
    } else {
      // phase 1: U = S Q_N (row strip) -> Bc = U^T [k_q][i_p];  V = S^T Q_{N-1} (column
      // strip) -> Bd = V^T [k_p][i_q]
      if (rowW) {
        f32x4 u[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        const u16* arow = Ss + (16 * wid + m16) * ldS + 8 * g4;
        for (int c = 0; c < ncq; ++c) {
          const bf16x8 av = frag_row(arow + 32 * c);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KqT) u[t] = mma16(av, frag_row(Bb + min(16 * t + m16, Kq - 1) * ldQ + 32 * c + 8 * g4), u[t]);
        }
        // C layout: lane holds U[16 wid + 4 g4 + r][16 t + m16]
#pragma unroll
        for (int t = 0; t < 2; ++t)
          if (t < KqT && 16 * t + m16 < Kq) {
            const int k = 16 * t + m16, i = 16 * wid + 4 * g4;
            const uint32_t lo = (uint32_t)bf16_bits(u[t][0]) | ((uint32_t)bf16_bits(u[t][1]) << 16);
            const uint32_t hi = (uint32_t)bf16_bits(u[t][2]) | ((uint32_t)bf16_bits(u[t][3]) << 16);
            *(uint2*)(Bc + k * ldP + i) = make_uint2(lo, hi);
          }
      }
      if (colW) {
        f32x4 v[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
        const u16* acol = Ss + (8 * g4 + (m16 >> 2)) * ldS + 16 * wid + 4 * (m16 & 3);
        for (int c = 0; c < ncp; ++c) {
          const bf16x8 av = frag_col_tr(acol + 32 * c * ldS, ldS);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KpT) v[t] = mma16(av, frag_row(Ba + min(16 * t + m16, Kp - 1) * ldP + 32 * c + 8 * g4), v[t]);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
          if (t < KpT && 16 * t + m16 < Kp) {
            const int k = 16 * t + m16, i = 16 * wid + 4 * g4;
            const uint32_t lo = (uint32_t)bf16_bits(v[t][0]) | ((uint32_t)bf16_bits(v[t][1]) << 16);
            const uint32_t hi = (uint32_t)bf16_bits(v[t][2]) | ((uint32_t)bf16_bits(v[t][3]) << 16);
            *(uint2*)(Bd + k * ldQ + i) = make_uint2(lo, hi);
          }
      }
      __syncthreads();
      // phase 2: Y'_{N-1}[strip rows] += S V;  Y'_N[strip cols] += S^T U
      if (rowW) {
        const u16* arow = Ss + (16 * wid + m16) * ldS + 8 * g4;
        for (int c = 0; c < ncq; ++c) {
          const bf16x8 av = frag_row(arow + 32 * c);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KpT) accp[t] = mma16(av, frag_row(Bd + min(16 * t + m16, Kp - 1) * ldQ + 32 * c + 8 * g4), accp[t]);
        }
      }
      if (colW) {
        const u16* acol = Ss + (8 * g4 + (m16 >> 2)) * ldS + 16 * wid + 4 * (m16 & 3);
        for (int c = 0; c < ncp; ++c) {
          const bf16x8 av = frag_col_tr(acol + 32 * c * ldS, ldS);
#pragma unroll
          for (int t = 0; t < 2; ++t)
            if (t < KqT) accq[t] = mma16(av, frag_row(Bc + min(16 * t + m16, Kq - 1) * ldP + 32 * c + 8 * g4), accq[t]);
        }
      }
    }
  }
  // this work-group's partials: rows 16 wid + 4 g4 + r, columns 16 t + m16
  if (rowW) {
    float* dst = p.partp + (int64_t)blockIdx.x * Ip * Kp;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = 16 * t + m16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * wid + 4 * g4 + r;
        if (t < KpT && i < Ip && k < Kp) dst[i * Kp + k] = accp[t][r];
      }
    }
  }
  if (colW) {
    float* dst = p.partq + (int64_t)blockIdx.x * Iq * Kq;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int k = 16 * t + m16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * wid + 4 * g4 + r;
        if (t < KqT && i < Iq && k < Kq) dst[i * Kq + k] = accq[t][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
namespace {

void slab_fill(SlabArgs& p, int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq) {
  p.A = A;
  p.Ip = (int)Ip;
  p.Iq = (int)Iq;
  p.Kp = Kp;
  p.Kq = Kq;
  p.nsp = (int)((Ip + 15) / 16);
  p.nsq = (int)((Iq + 15) / 16);
  // pitches: multiples of 8 (16-byte fragment reads) covering the 32-wide chunks
  p.ldS = (int)((Iq + 31) / 32 * 32 + 8);
  p.ldP = (int)((Ip + 31) / 32 * 32 + 8);
  p.ldQ = (int)((Iq + 31) / 32 * 32 + 8);
}

int slab_threads(const SlabArgs& p) { return 64 * (p.nsp > p.nsq ? p.nsp : p.nsq); }

size_t slab_lds(const SlabArgs& p, int op) { return (size_t)SlabLayout(p, op).total * 2; }

}  // namespace

bool slab_pass_supported(int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq, const void* X,
                         int op) {
  if (Ip < 16 || Iq < 16 || Ip > kSbMaxI || Iq > kSbMaxI || Iq % 4 != 0) return false;
  if (Kp < 1 || Kq < 1 || Kp > kSbMaxK || Kq > kSbMaxK || Kp >= Ip || Kq >= Iq) return false;
  if (((uintptr_t)X & 15) != 0 || A < 256) return false;
  SlabArgs p{};
  slab_fill(p, A, Ip, Iq, Kp, Kq);
  const int nth = slab_threads(p);
  if ((int64_t)Ip * Iq / 4 > (int64_t)kSbLoads * nth) return false;  // register staging
  return slab_lds(p, op) <= 150 * 1024;
}

int64_t slab_pass_grid(int64_t A) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipGetLastError();
  return A < cus ? A : cus;
}

hipError_t launch_slab_pass(int op, const void* X, int64_t A, int64_t Ip, int64_t Iq, int Kp,
                            int Kq, uint64_t seed, uint32_t swp, uint32_t swq, uint32_t tensor_id,
                            const double* Qp, const double* Qq, float* partp, float* partq,
                            int64_t grid, hipStream_t s) {
  SlabArgs p{};
  slab_fill(p, A, Ip, Iq, Kp, Kq);
  p.X = (const float*)X;
  p.seed = seed;
  p.swp = swp;
  p.swq = swq;
  p.tid = tensor_id;
  p.Qp = Qp;
  p.Qq = Qq;
  p.partp = partp;
  p.partq = partq;
  const bool l13 = (int64_t)Ip * Iq / 4 <= 13LL * slab_threads(p);
  const void* fn = op == 0 ? (l13 ? (const void*)slab_pass_kernel<0, 13> : (const void*)slab_pass_kernel<0, 16>)
                           : (l13 ? (const void*)slab_pass_kernel<1, 13> : (const void*)slab_pass_kernel<1, 16>);
  const size_t lds = slab_lds(p, op);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin(op == 0 ? "sketch_slab" : "power_slab", s);
  void* args[] = {&p};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(slab_threads(p)), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
