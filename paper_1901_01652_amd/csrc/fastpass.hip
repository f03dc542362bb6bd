// Persistent matrix-core passes over X for one mode n (FP32 input):
//   sketch  Y_n  += T M      (Alg. 1 steps 4-5; M drawn on the fly, never stored)
//   power   Y'_n += T (T^T Q_n)   (one round of subspace iteration, fiber form)
// where T is a tile of 64 consecutive columns of X_(n) with all I_n rows.  The sketch of a mode
// longer than 256 runs as several launches over row blocks of at most 256 rows each: rows of
// Y_n depend only on the same rows of X_(n), and every block draws the same M (keyed by j, k).
// Likewise a projection size above 64 runs as column blocks of at most 64: columns of Y_n (and
// of the power step's X_(n) X_(n)^T Q_n) depend only on the same columns of M (of Q_n).
//
// Tiles: column j of X_(n) is (a, b) with j = a*B + b for X viewed as A x I_n x B, so a
// tile of consecutive j is one or more contiguous runs of each row.  Three loaders:
//   cols4   B % 4 == 0: 16-byte loads along b (covers runs that cross an a boundary)
//   last4   B == 1 (mode N) and I_n % 4 == 0: 16-byte loads along the fiber itself
//   scalar  anything else.
// The tile is staged through registers (the next tile's loads are in flight while the
// matrix cores work on the current one) into LDS as bf16 (BF16 path, round to nearest
// even) or FP32.  Each work-group keeps its share of Y in accumulators across all its
// tiles and writes one partial at the end; reduce_partials sums them in a fixed order.
//
// LDS (BF16 path, I_n = 200, K = 20): T [I_n][64+8], M^T or W^T [K][64+8], and for the
// power step T^T [64][I_n+pad] and Q^T [K][I_n+pad].  The contraction index of every
// operand is contiguous, so each lane reads its 8 bf16 with one 16-byte LDS access.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

constexpr int kFpTJ = 64;

// Column of element (row, col) of the [i][j] tile for the contiguous-fiber loader: the 8-wide
// column groups of a row are XOR-permuted by (row / 16) mod 8.  That loader's threads write
// four consecutive rows of one column, which without the permutation land in 4 of the 64 LDS
// banks (16-way conflicts); the permutation spreads them, and 8-element groups stay whole so
// the matrix-core reads below remain single 16-byte loads.
__device__ __forceinline__ int swz_col(int row, int col) {
  return ((((col >> 3) ^ (row >> 4)) & 7) << 3) | (col & 7);
}
constexpr int kFpThreads = 512;   // 8 wavefronts

__device__ __forceinline__ uint32_t bf16_u16(float v) {
  const __bf16 b = (__bf16)v;
  return (uint32_t)*(const unsigned short*)&b;
}
constexpr int kFpMaxIn = 256;
constexpr int kFpMaxK = 64;

struct PassArgs {
  const float* X;    // first element of the row block
  int64_t A, In, B, J;
  int64_t strideA;   // elements between consecutive a (the full mode's I_n * B)
  int Ktot, k0;      // column block [k0, k0 + K) of a projection of size Ktot
  KrArgs kr;         // kr.f != nullptr: Khatri-Rao test matrix (FP32 factors)
  int K;
  uint64_t seed;
  uint32_t stream, tid;
  const double* Q;  // power step: In x K row-major
  int64_t ntiles;
  float* partial;   // [gridDim.x][In][K]
  int loader;       // 0 cols4, 1 last4, 2 scalar
  int ldT, ldI, kI; // LDS leading dimensions, padded contraction length over i
};

template <int PR>
struct PassLds {
  using T = typename Mma<PR>::T;
  static __host__ __device__ int mt_pad(int64_t In) { return (int)((In + 15) / 16) * 16; }
  static __host__ __device__ int kt_pad(int K) { return ((K + 15) / 16) * 16; }
};

// Layout of the dynamic LDS block (element offsets in T units, 16-byte aligned).
template <int PR, int OP>
struct PassLayout {
  using T = typename Mma<PR>::T;
  int oTij, oOt, oTji, oQt, total;
  __host__ __device__ PassLayout(int64_t In, int K, int ldT, int ldI) {
    const int a = 16 / (int)sizeof(T);
    auto up = [a](int v) { return (v + a - 1) / a * a; };
    // bf16 power step: no transposed copy (its products read the row-major tile with
    // transposing loads), and the tile spans whole 32-row contraction chunks (zero rows)
    constexpr bool tr = OP == 1 && PR == 1;
    const int MTp = tr ? (int)((In + 31) / 32) * 32 : (int)((In + 15) / 16) * 16;
    const int KTp = ((K + 15) / 16) * 16;
    oTij = 0;
    oOt = up(oTij + MTp * ldT);
    oTji = up(oOt + KTp * ldT);
    oQt = up(oTji + (OP == 1 && !tr ? kFpTJ * ldI : 0));
    total = up(oQt + (OP == 1 ? KTp * ldI : 0));
  }
};

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// One 16 x 16 tile of W^T = Q^T T for the bf16 power step: A = rows of Q^T (contraction index
// i contiguous, pitch ldq), B = column block jt of the row-major tile T [i][j] (pitch ldt, the
// 8-column groups permuted as in swz_col when LD == 1), read with transposing LDS loads
// (ds_read_b64_tr_b16) instead of from a transposed copy.  In each 16-lane block the load
// gives lane 4 q + e element e of the 8-byte row runs named by lanes q, q + 4, q + 8, q + 12,
// so lane 16 g + r names row 8 g + (r >> 2) (and + 4), columns 16 jt + 4 (r & 3) .. + 3, and
// receives T[8 g .. 8 g + 7][16 jt + r], the B operand.  Blocks with g odd read their upper
// four rows first: with a pitch of 36 words the eight rows of a 32-lane read then fall on
// disjoint banks; their halves come back swapped and are put in order with a select.
template <int LD>
__device__ __forceinline__ f32x4 wt_tile_tr(const __bf16* Qt, int ldq, const __bf16* Tij, int ldt,
                                            int jt, int kdim) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const bool up = (g & 1) != 0;
  const __bf16* a = Qt + r * ldq + 8 * g;
  const int r0 = 8 * g + (r >> 2) + (up ? 4 : 0), r1 = r0 + (up ? -4 : 4);
  const int c = 16 * jt + 4 * (r & 3);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < kdim; k += 32) {
    const int ra = k + r0, rb = k + r1;
    const int ca = LD == 1 ? swz_col(ra, c) : c, cb = LD == 1 ? swz_col(rb, c) : c;
    const s16x4 x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(Tij + ra * ldt + ca));
    const s16x4 y = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(Tij + rb * ldt + cb));
    union {
      s16x4 h[2];
      bf16x8 v;
    } u;
    u.h[0] = up ? y : x;
    u.h[1] = up ? x : y;
    const bf16x8 av = *(const bf16x8*)(a + k);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, u.v, acc, 0, 0, 0);
  }
  return acc;
}

// AQ: 16x16 output tiles of Y per wavefront (4 covers In <= 128 x K <= 64 or In <= 256 x
// K <= 32, 8 the rest).  With the 16-byte loader and AQ = 4 the kernel is held to 128 VGPRs
// (4 waves per SIMD: two work-groups per CU, twice the loads in flight); the other variants
// would spill at that cap.
template <int PR, int OP, int LD, int AQ>
__global__ __launch_bounds__(kFpThreads, (LD == 0 && AQ == 4 ? 4 : 2)) void mode_pass_kernel(PassArgs p) {
  using T = typename Mma<PR>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = (T*)smem_raw;
  const PassLayout<PR, OP> L(p.In, p.K, p.ldT, p.ldI);
  T* Tij = smem + L.oTij;
  T* Ot = smem + L.oOt;  // M^T (sketch) or W^T (power), [k][j]
  T* Tji = smem + L.oTji;
  T* Qt = smem + L.oQt;
  const int In = (int)p.In, K = p.K, ldT = p.ldT, ldI = p.ldI;
  const int MT = (In + 15) / 16, NT = (K + 15) / 16;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;  // 8 waves

  for (int x = tid; x < L.total; x += kFpThreads) smem[x] = Mma<PR>::cvt(0.f);
  __syncthreads();
  if (OP == 1) {
    for (int x = tid; x < In * K; x += kFpThreads) {
      const int i = x / K, k = x % K;
      Qt[k * ldI + i] = Mma<PR>::cvt((float)p.Q[(int64_t)i * p.Ktot + p.k0 + k]);
    }
  }

  f32x4 acc[AQ];  // output tiles q = wid + 8 s of the (MT x NT) grid
#pragma unroll
  for (int s = 0; s < AQ; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

  float4 buf[8];
  auto load = [&](int64_t t) {
    const int64_t j0 = t * kFpTJ;
    if constexpr (LD == 0) {
      const int c4 = tid & 15;
      const int64_t j = j0 + 4 * c4;
      const bool ok = j < p.J;
      const int64_t cb = ok ? (j / p.B) * p.strideA + (j % p.B) : 0;
      // one per-lane base; the step between the eight rows is uniform, so the eight
      // addresses do not each hold a register pair across the tile loop
      const float* xb = p.X + cb + (int64_t)(tid >> 4) * p.B;
      const int64_t rs = 32 * p.B;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int i = (tid >> 4) + 32 * s;
        buf[s] = (ok && i < In) ? *(const float4*)(xb + s * rs) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else if constexpr (LD == 1) {
      const int q4 = In / 4;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int f = tid + kFpThreads * s;
        const int al = f / q4, i4 = f % q4;
        const int64_t j = j0 + al;
        buf[s] = (al < kFpTJ && j < p.J) ? *(const float4*)(p.X + j * p.strideA + 4 * i4)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      const int jl = tid & 63;
      const int64_t j = j0 + jl;
      const bool ok = j < p.J;
      const int64_t cb = ok ? (j / p.B) * p.strideA + (j % p.B) : 0;
#pragma unroll
      for (int s = 0; s < 32; ++s) {
        const int i = (tid >> 6) + 8 * s;
        const float v = (ok && i < In) ? p.X[cb + (int64_t)i * p.B] : 0.f;
        if ((s & 3) == 0) buf[s >> 2].x = v;
        if ((s & 3) == 1) buf[s >> 2].y = v;
        if ((s & 3) == 2) buf[s >> 2].z = v;
        if ((s & 3) == 3) buf[s >> 2].w = v;
      }
    }
  };
  auto store = [&]() {
    if constexpr (LD == 0) {
      const int c4 = tid & 15;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int i = (tid >> 4) + 32 * s;
        const float4 v = buf[s];
        if constexpr (PR == 1) {
          // the four values as two bf16 pairs, stored to the row-major tile as one 8-byte word
          // (ldT is a multiple of 4 elements)
          const uint32_t p01 = (uint32_t)bf16_u16(v.x) | ((uint32_t)bf16_u16(v.y) << 16);
          const uint32_t p23 = (uint32_t)bf16_u16(v.z) | ((uint32_t)bf16_u16(v.w) << 16);
          if (i < In) *(uint2*)(Tij + i * ldT + 4 * c4) = make_uint2(p01, p23);
        } else {
          if (i < In) {
            T* d = Tij + i * ldT + 4 * c4;
            d[0] = Mma<PR>::cvt(v.x);
            d[1] = Mma<PR>::cvt(v.y);
            d[2] = Mma<PR>::cvt(v.z);
            d[3] = Mma<PR>::cvt(v.w);
          }
          if (OP == 1 && i < In) {
            Tji[(4 * c4 + 0) * ldI + i] = Mma<PR>::cvt(v.x);
            Tji[(4 * c4 + 1) * ldI + i] = Mma<PR>::cvt(v.y);
            Tji[(4 * c4 + 2) * ldI + i] = Mma<PR>::cvt(v.z);
            Tji[(4 * c4 + 3) * ldI + i] = Mma<PR>::cvt(v.w);
          }
        }
      }
    } else if constexpr (LD == 1) {
      const int q4 = In / 4;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int f = tid + kFpThreads * s;
        const int al = f / q4, i4 = f % q4;
        if (al < kFpTJ) {
          const float4 v = buf[s];
          const int i = 4 * i4;
          Tij[(i + 0) * ldT + swz_col(i + 0, al)] = Mma<PR>::cvt(v.x);
          Tij[(i + 1) * ldT + swz_col(i + 1, al)] = Mma<PR>::cvt(v.y);
          Tij[(i + 2) * ldT + swz_col(i + 2, al)] = Mma<PR>::cvt(v.z);
          Tij[(i + 3) * ldT + swz_col(i + 3, al)] = Mma<PR>::cvt(v.w);
          if (OP == 1 && PR != 1) {
            T* d = Tji + al * ldI + i;
            d[0] = Mma<PR>::cvt(v.x);
            d[1] = Mma<PR>::cvt(v.y);
            d[2] = Mma<PR>::cvt(v.z);
            d[3] = Mma<PR>::cvt(v.w);
          }
        }
      }
    } else {
      const int jl = tid & 63;
#pragma unroll
      for (int s = 0; s < 32; ++s) {
        const int i = (tid >> 6) + 8 * s;
        if (i < In) {
          const float4 v4 = buf[s >> 2];
          const float v = (s & 3) == 0 ? v4.x : (s & 3) == 1 ? v4.y : (s & 3) == 2 ? v4.z : v4.w;
          Tij[i * ldT + jl] = Mma<PR>::cvt(v);
          if (OP == 1 && PR != 1) Tji[jl * ldI + i] = Mma<PR>::cvt(v);
        }
      }
    }
  };
  // Khatri-Rao test matrix: thread (jl, g) forms column jl's factor rows once and the
  // products for k = g, g + 8, ..
  auto draw_kr = [&](int64_t t) {
    const int jl = tid & 63, g = tid >> 6;
    const int64_t j = t * kFpTJ + jl;
    const float* F = (const float*)p.kr.f;
    const int nm = p.kr.nm;
    int64_t row[7];
    int64_t r = j < p.J ? j : 0;
#pragma unroll
    for (int m = 6; m >= 0; --m) {
      if (m < nm) {
        const int d = p.kr.dim[m];
        const int64_t i = r % d;
        r /= d;
        row[m] = p.kr.off[m] + i * p.kr.ld + p.k0;
      }
    }
    for (int k = g; k < K; k += kFpThreads / 64) {
      float v = 1.f;
#pragma unroll
      for (int m = 0; m < 7; ++m)
        if (m < nm) v *= F[row[m] + k];
      Ot[k * ldT + jl] = Mma<PR>::cvt(j < p.J ? v : 0.f);
    }
  };
  // Column block of M for the tile's columns: row j holds stream elements
  // [j Ktot + k0, j Ktot + k0 + K); each thread takes one Philox call of one row
  auto draw_block = [&](int64_t t) {
    const int64_t j0 = t * kFpTJ;
    const int jvalid = (int)min((int64_t)kFpTJ, p.J - j0);
    const int cpr = K / 4 + 2;  // calls that can touch one row's K elements
    for (int x = tid; x < kFpTJ * cpr; x += kFpThreads) {
      const int jl = x / cpr, c = x % cpr;
      const int64_t es = (j0 + jl) * p.Ktot + p.k0;
      const int64_t call = (es >> 2) + c;
      float z[4];
      normals4(p.seed, p.stream, p.tid, (uint64_t)call, z);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int64_t k = 4 * call + l - es;
        if (k >= 0 && k < K) Ot[k * ldT + jl] = Mma<PR>::cvt(jl < jvalid ? z[l] : 0.f);
      }
    }
  };
  // Rows of M for the tile's columns: stream elements [j0*K, (j0+64)*K), written M^T[k][jl].
  auto draw = [&](int64_t t) {
    const int64_t j0 = t * kFpTJ;
    const int64_t e0 = j0 * K;
    const int span = kFpTJ * K;  // stream elements of the tile, < 2^12
    const int jvalid = (int)min((int64_t)kFpTJ, p.J - j0);
    const int64_t c0 = e0 >> 2;
    const int off = (int)(e0 - 4 * c0);  // position of e0 inside its call (0..3)
    const int ncalls = (off + span + 3) >> 2;
    for (int ci = tid; ci < ncalls; ci += kFpThreads) {
      float z[4];
      normals4(p.seed, p.stream, p.tid, (uint64_t)(c0 + ci), z);
      const int rel = 4 * ci - off;        // offset of lane 0 from e0 (negative only for ci = 0)
      const int l0 = rel < 0 ? -rel : 0;   // first lane inside the tile
      int jl = (rel + l0) / K;
      int k = (rel + l0) - jl * K;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        if (l >= l0) {
          if (rel + l < span) Ot[k * ldT + jl] = Mma<PR>::cvt(jl < jvalid ? z[l] : 0.f);
          if (++k == K) {
            k = 0;
            ++jl;
          }
        }
      }
    }
  };

  // XCD-aware order: work-groups are dealt round-robin to the 8 XCDs, so block b runs on
  // XCD b % 8.  Renumber them so that each XCD takes a contiguous run of tiles per round;
  // neighbouring tiles share the cache lines at their boundaries (rows that are not
  // 128-byte aligned), and those lines are then fetched into one L2 instead of two.
  const int64_t G = gridDim.x;
  int64_t t = (G % 8 == 0) ? (int64_t)(blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  if (t < p.ntiles) load(t);
  for (; t < p.ntiles; t += gridDim.x) {
    store();
    if (OP == 0) {
      if (p.kr.f)
        draw_kr(t);
      else if (p.Ktot == K)
        draw(t);
      else
        draw_block(t);
    }
    __syncthreads();
    const int64_t tn = t + gridDim.x;
    if (tn < p.ntiles) load(tn);
    if (OP == 1) {
      // W^T [K x 64] = Q^T [K x In] * T [In x 64]  (contraction over i)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int q = wid + 8 * s;
        if (q < NT * 4) {
          const int nt = q >> 2, jt = q & 3;
          f32x4 w;
          if constexpr (PR == 1)
            w = wt_tile_tr<LD>(Qt + nt * 16 * ldI, ldI, Tij, ldT, jt, p.kI);
          else
            w = tile_abt(Qt + nt * 16 * ldI, ldI, Tji + jt * 16 * ldI, ldI, p.kI,
                         f32x4{0.f, 0.f, 0.f, 0.f});
          const int col = jt * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) Ot[(nt * 16 + 4 * (lane >> 4) + r) * ldT + col] = Mma<PR>::cvt(w[r]);
        }
      }
      __syncthreads();
    }
    // Y [In x K] += T [In x 64] * (M or W) [64 x K]
#pragma unroll
    for (int s = 0; s < AQ; ++s) {
      const int q = wid + 8 * s;
      if (q < MT * NT) {
        const int mt = q / NT, nt = q % NT;
        if constexpr (LD == 1) {
          // tile_abt with the swizzled A operand: lane reads row mt*16 + (lane & 15),
          // column group (k0 / 8 + lane / 16) permuted as in swz_col
          const int r = mt * 16 + (lane & 15), gq = lane >> 4;
          const T* arow = Tij + r * ldT;
          const T* brow = Ot + (nt * 16 + (lane & 15)) * ldT;
          f32x4 c = acc[s];
          if constexpr (PR != 0) {
            using V8 = typename Mma<PR>::V8;
#pragma unroll
            for (int k0 = 0; k0 < kFpTJ; k0 += 32) {
              const int ca = swz_col(r, k0 + 8 * gq);
              const V8 av = *(const V8*)(arow + ca);
              const V8 bv = *(const V8*)(brow + k0 + 8 * gq);
              c = Mma<PR>::mma8(av, bv, c);
            }
          } else {
#pragma unroll
            for (int k0 = 0; k0 < kFpTJ; k0 += 4)
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(arow[swz_col(r, k0 + gq)],
                                                      brow[k0 + gq], c, 0, 0, 0);
          }
          acc[s] = c;
        } else {
          acc[s] = tile_abt(Tij + mt * 16 * ldT, ldT, Ot + nt * 16 * ldT, ldT, kFpTJ, acc[s]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < AQ; ++s) {
    const int q = wid + 8 * s;
    if (q < MT * NT) {
      const int mt = q / NT, nt = q % NT;
      const int n = nt * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mt * 16 + 4 * (lane >> 4) + r;
        if (m < In && n < K) p.partial[((int64_t)blockIdx.x * In + m) * K + n] = acc[s][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Operand precision of an arithmetic: 0 FP32, 1 bf16, 2 fp8 (e4m3).
static int prec_of(Arith ar) { return ar == kBF16 ? 1 : ar == kFP8 ? 2 : 0; }
static int ld_t(int pr) { return pr ? kFpTJ + 8 : kFpTJ + 2; }
static int k_i(int pr, int64_t In) { return pr ? (int)((In + 31) / 32 * 32) : (int)((In + 3) / 4 * 4); }
static int ld_i(int pr, int64_t In) { return k_i(pr, In) + (pr ? 8 : 2); }

// Output tiles per wavefront needed for an In x K result over 8 wavefronts.
static int acc_slots(int64_t In, int K) {
  const int64_t tiles = ((In + 15) / 16) * ((K + 15) / 16);
  return tiles <= 32 ? 4 : 8;
}

static size_t pass_lds(int pr, int op, int64_t In, int K) {
  const int ldT = ld_t(pr), ldI = ld_i(pr, In);
  int total;
  if (pr == 1)
    total = op ? PassLayout<1, 1>(In, K, ldT, ldI).total : PassLayout<1, 0>(In, K, ldT, ldI).total;
  else if (pr == 2)
    total = op ? PassLayout<2, 1>(In, K, ldT, ldI).total : PassLayout<2, 0>(In, K, ldT, ldI).total;
  else
    total = op ? PassLayout<0, 1>(In, K, ldT, ldI).total : PassLayout<0, 0>(In, K, ldT, ldI).total;
  return (size_t)total * (pr == 1 ? 2 : pr == 2 ? 1 : 4);
}

constexpr size_t kFpLdsMax = 160 * 1024;

// Widest column block (64, 48, 32 or 16, or K itself when smaller) whose LDS layout fits;
// 0 when the pass does not take this mode.
int fast_pass_block_k(Arith ar, const ModeView& v, int K, int op) {
  if (ar == kF64 || K < 1 || (ar == kFP8 && op != 0)) return 0;  // fp8: the sketch only
  int64_t rows = v.In;
  if (v.In > kFpMaxIn) {  // the sketch in row blocks; the power step needs every row at once
    if (op != 0) return 0;
    rows = kFpMaxIn;
  }
  const int widths[4] = {kFpMaxK, 48, 32, 16};
  for (int w : widths) {
    const int kb = K < w ? K : w;
    if (pass_lds(prec_of(ar), op, rows, kb) <= kFpLdsMax) return kb;
  }
  return 0;
}

bool fast_pass_supported(Arith ar, const ModeView& v, int K, int op) {
  return fast_pass_block_k(ar, v, K, op) > 0;
}

int64_t fast_pass_block_rows() { return kFpMaxIn; }

static const void* pass_fn(int pr, int op, int loader, int aq) {
#define RTR_FP_SEL(P_, O_, L_) \
  if (pr == P_ && op == O_ && loader == L_)                                        \
    return aq == 4 ? (const void*)mode_pass_kernel<P_, O_, L_, 4>                  \
                   : (const void*)mode_pass_kernel<P_, O_, L_, 8>;
  RTR_FP_SEL(1, 0, 0) RTR_FP_SEL(1, 0, 1) RTR_FP_SEL(1, 0, 2)
  RTR_FP_SEL(1, 1, 0) RTR_FP_SEL(1, 1, 1) RTR_FP_SEL(1, 1, 2)
  RTR_FP_SEL(0, 0, 0) RTR_FP_SEL(0, 0, 1) RTR_FP_SEL(0, 0, 2)
  RTR_FP_SEL(0, 1, 0) RTR_FP_SEL(0, 1, 1) RTR_FP_SEL(0, 1, 2)
  RTR_FP_SEL(2, 0, 0) RTR_FP_SEL(2, 0, 1) RTR_FP_SEL(2, 0, 2)
#undef RTR_FP_SEL
  return nullptr;
}

// X: first element of the row block; strideA: the full mode's I_n * B.
static int pick_loader(const void* X, const ModeView& v, int64_t strideA) {
  const bool al16 = ((uintptr_t)X & 15) == 0;
  if (al16 && v.B % 4 == 0) return 0;
  if (al16 && v.B == 1 && v.In % 4 == 0 && strideA % 4 == 0) return 1;
  return 2;
}

// The row block [row0, row0 + rows) of X_(n) as a mode view of its own (rows = 0: all).
static ModeView block_view(const ModeView& v, int64_t row0, int64_t rows) {
  ModeView b = v;
  b.In = rows > 0 ? rows : v.In - row0;
  return b;
}

// Work-groups resident per CU (HIP occupancy query) times the CU count.
int64_t fast_pass_grid(Arith ar, const ModeView& v, int K, int op, const void* X, int64_t row0,
                       int64_t rows) {
  const int pr = prec_of(ar);
  const ModeView b = block_view(v, row0, rows);
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + kFpTJ - 1) / kFpTJ;
  const size_t lds = pass_lds(pr, op, b.In, K);
  const void* fn = pass_fn(pr, op, pick_loader((const float*)X + row0 * v.B, b, v.In * v.B),
                           acc_slots(b.In, K));
  if (!fn) return 0;
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kFpThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  (void)hipGetLastError();
  const int64_t g = (int64_t)cus * per_cu;
  return ntiles < g ? ntiles : g;
}

hipError_t launch_fast_pass(Arith ar, int op, const void* X, const ModeView& v, int K,
                            uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                            const double* Q, void* partial, int64_t grid, hipStream_t s,
                            int64_t row0, int64_t rows, int Ktot, int k0, const KrArgs* kr) {
  if (Ktot == 0) Ktot = K;
  if (k0 < 0 || K < 1 || K > kFpMaxK || k0 + K > Ktot) return hipErrorInvalidValue;
  const int pr = prec_of(ar);
  const ModeView b = block_view(v, row0, rows);
  if (row0 < 0 || b.In < 1 || row0 + b.In > v.In || b.In > kFpMaxIn || (op != 0 && b.In != v.In))
    return hipErrorInvalidValue;
  PassArgs p{};
  p.X = (const float*)X + row0 * v.B;
  p.A = v.A;
  p.In = b.In;
  p.B = v.B;
  p.strideA = v.In * v.B;
  p.J = v.A * v.B;
  p.K = K;
  p.Ktot = Ktot;
  p.k0 = k0;
  if (kr) p.kr = *kr;
  p.seed = seed;
  p.stream = stream_word;
  p.tid = tensor_id;
  p.Q = Q;
  p.ntiles = (p.J + kFpTJ - 1) / kFpTJ;
  p.partial = (float*)partial;
  p.loader = pick_loader(p.X, b, p.strideA);
  p.ldT = ld_t(pr);
  p.ldI = ld_i(pr, b.In);
  p.kI = k_i(pr, b.In);
  const size_t lds = pass_lds(pr, op, b.In, K);
  const void* fn = pass_fn(pr, op, p.loader, acc_slots(b.In, K));
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin(op ? "power_fused" : "sketch_fused", s);
  void* args[] = {&p};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kFpThreads), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
