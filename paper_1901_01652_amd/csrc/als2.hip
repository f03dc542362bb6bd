// TR-ALS (Alg. 1 step 9) with two kernels per core update.
//
// Core n is the least-squares solution of Eq. (2) restricted to P:
//   P_<n> ~ Z_{n,(2)} B^T,  B[j, a*R_{n+1} + b] = S_j[b, a],
//   S_j = Z_{n+1}(i_{n+1}) ... Z_N(i_N) Z_1(i_1) ... Z_{n-1}(i_{n-1}),
// through the normal equations Gram * Z_{n,(2)}^T = M^T with M = P_<n> B, Gram = B^T B.
//
// als_accum  one tile of TJ columns j per pass: the tile's subchain rows are formed in LDS
//            (one row b of S_j per thread: the first slice row is copied, the other cores
//            are vector-matrix products), then M += P_<n>[:, tile] B_tile (and B^T B when the
//            Gram is accumulated directly) on the FP64 matrix cores.  Optionally the same
//            tile gives ||P - Psi(Z)||^2 with the current core n, so the first update of a
//            sweep reports the error of the sweep before it without another pass.
// als_solve  one work-group: fixed-order sum of the partials; Gram from transfer matrices
//            E_m = sum_i Z_m(i) (x) Z_m(i) multiplied around the ring (FP64 matrix cores)
//            when every rank is small; the normal equations solved in FP64 by Gauss-Jordan
//            elimination without pivoting on [Gram | M^T] (solve.hpp: every pivot of a
//            positive-definite Gram is a positive Schur-complement diagonal, so this gives
//            the Cholesky solution; a non-positive pivot is the failure flag); the new core.
//            Cholesky with forward and back substitution remains only as the fallback for
//            systems too large for the Gauss-Jordan register tiers.  It also closes the previous sweep (error, stopping test, and
//            the device flag that turns every later kernel of the decomposition into a no-op).
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"
#include "solve.hpp"

namespace rtr {

constexpr int kAcThreads = 1024;  // 16 wavefronts
constexpr int kSolveThreads = 1024;
constexpr int kAcTilesMax = 8;    // 16x16 output tiles per wavefront, at most
constexpr int64_t kZldsMax = 6144;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static __host__ __device__ inline int pad16(int v) { return (v + 15) / 16 * 16; }
static __host__ __device__ inline int64_t zwords(int64_t z) { return (z + 1) / 2 * 2; }

// ---------------------------------------------------------------------------------------
__device__ void transfer_gram(const double* __restrict__ Z, int64_t ztotal, int N, int n,
                              const int64_t* zoff, const int* Kc, const int* Rc, int tdim, int Ra,
                              int Rb, double* xt, double* G, const double* Zstaged = nullptr);

template <int RM, int TJ, int kAcTiles>
__global__ __launch_bounds__(kAcThreads) void als_accum_kernel(AlsArgs2 g) {
  extern __shared__ __align__(16) double sm[];
  if (g.gram_extra && blockIdx.x == gridDim.x - 1) {  // the Gram, beside the accumulation
    if (*g.done) return;
    transfer_gram(g.Z, g.ztotal, g.N, g.n, g.zoffs, g.Kc, g.Rc, g.tdim, g.Ra, g.Rb, sm,
                  g.gram_out);
    return;
  }
  const int RR = g.RR, Kn = g.Kn, Ra = g.Ra, Rb = g.Rb;
  const int NT = pad16(RR) / 16, MT = pad16(Kn) / 16;
  const int ldB = pad16(RR) + 1, ldL = TJ + 1;
  double* Zs = sm;
  double* Bs = sm + (g.zlds ? zwords(g.ztotal) : 0);  // [TJ][ldB]
  double* Ls = Bs + TJ * ldB;                          // [pad16(Kn)][ldL]
  const double* Zsrc = g.zlds ? Zs : g.Z;
  __shared__ double red[32];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (g.zlds) {  // cores: every load issued before any store
    double zt[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int64_t x = tid + (int64_t)e * kAcThreads;
      zt[e] = x < g.ztotal ? g.Z[x] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int64_t x = tid + (int64_t)e * kAcThreads;
      if (x < g.ztotal) Zs[x] = zt[e];
    }
  }
  for (int x = tid; x < TJ * ldB; x += kAcThreads) Bs[x] = 0.0;  // padding columns stay 0
  if (*g.done) return;
  const int nM = Kn * RR;
  const int ntM = MT * NT, ntot = ntM + (g.gram_direct ? NT * NT : 0);
  const bool accum = g.mode & 1, resid = g.mode & 2;
  f64x4 acc[kAcTiles];
#pragma unroll
  for (int s = 0; s < kAcTiles; ++s) acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
  double rsum = 0.0;
  const int64_t ntiles = (g.J + TJ - 1) / TJ;
  const int64_t t0 = (int64_t)blockIdx.x * g.tiles_per_wg;
  const int64_t t1 = min(ntiles, t0 + g.tiles_per_wg);
  for (int64_t t = t0; t < t1; ++t) {
    const int j0 = (int)(t * TJ);
    const int jn = (int)min((int64_t)TJ, g.J - j0);
    __syncthreads();
    // P_<n>[:, tile] into Ls (rows padded to a multiple of 16 with zeros), 64 rows at a time
    for (int i0 = 0; i0 < MT * 16; i0 += 64) {
      constexpr int kPer = (64 * TJ + kAcThreads - 1) / kAcThreads;
      double pv[kPer];
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int x = tid + e * kAcThreads;
        const int i = i0 + x / TJ, jj = x % TJ;
        pv[e] = 0.0;
        if (i < Kn && jj < jn) {
          int rem = j0 + jj, base = 0;
#pragma unroll
          for (int u = 6; u >= 0; --u) {
            if (u <= g.N - 2) {
              const int d = g.cycK[u];
              const int q = rem / d;
              base += (rem - q * d) * (int)g.cycStride[u];
              rem = q;
            }
          }
          pv[e] = g.P[base + i * (int)g.strideN];
        }
      }
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int x = tid + e * kAcThreads;
        const int i = i0 + x / TJ, jj = x % TJ;
        if (x < 64 * TJ && i < MT * 16) Ls[i * ldL + jj] = pv[e];
      }
    }
    // subchain rows: thread (jl, b) forms row b of S_j
    for (int x = tid; x < TJ * Rb; x += kAcThreads) {
      const int jl = x / Rb, b = x % Rb;
      double v[RM], w[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = 0.0;
      if (jl < jn) {
        int rem = j0 + jl;
        int idx[7];
#pragma unroll
        for (int u = 6; u >= 0; --u) {
          if (u <= g.N - 2) {
            idx[u] = rem % g.chI[u];
            rem /= g.chI[u];
          }
        }
        // first core: row b of its slice
        {
          const int cRb = g.chRb[0];
          const double* G0 = Zsrc + g.chOff[0] + ((int64_t)b * g.chI[0] + idx[0]) * cRb;
#pragma unroll
          for (int c = 0; c < RM; ++c) v[c] = c < cRb ? G0[c] : 0.0;
        }
        int cur = g.chRb[0];
#pragma unroll
        for (int u = 1; u < 7; ++u) {
          if (u < g.N - 1) {
            const int cRb = g.chRb[u];
            const double* G = Zsrc + g.chOff[u] + (int64_t)idx[u] * cRb;
            const int rs = g.chI[u] * cRb;
#pragma unroll
            for (int c = 0; c < RM; ++c) w[c] = 0.0;
#pragma unroll
            for (int a = 0; a < RM; ++a) {
              if (a < cur) {
                const double va = v[a];
                const double* gr = G + a * rs;
#pragma unroll
                for (int c = 0; c < RM; ++c)
                  if (c < cRb) w[c] += va * gr[c];
              }
            }
#pragma unroll
            for (int c = 0; c < RM; ++c) v[c] = w[c];
            cur = cRb;
          }
        }
      }
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < Ra) Bs[jl * ldB + a * Rb + b] = v[a];
    }
    __syncthreads();
    if (accum) {
      const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
      for (int s = 0; s < kAcTiles; ++s) {
        const int q = wid + 16 * s;
        if (q < ntot) {
          const double* ap;
          int ast;  // A(m, k) = ap[k * ast] for this lane's row m
          int nt;
          if (q < ntM) {
            const int mt = q / NT;
            nt = q % NT;
            ap = Ls + (mt * 16 + r16) * ldL + g4;  // A = P tile (rows i, contraction j)
            ast = 1;
          } else {
            const int qq = q - ntM;
            const int mt = qq / NT;
            nt = qq % NT;
            ap = Bs + g4 * ldB + mt * 16 + r16;  // A = B^T (rows r1, contraction j)
            ast = ldB;
          }
          const double* bp = Bs + g4 * ldB + nt * 16 + r16;
          f64x4 c = acc[s];
#pragma unroll 8
          for (int k0 = 0; k0 < TJ; k0 += 4) c = mma_f64(ap[k0 * ast], bp[k0 * ldB], c);
          acc[s] = c;
        }
      }
    }
    if (resid) {
      const double* Zn = Zsrc + g.zoffN;
      for (int x = tid; x < Kn * TJ; x += kAcThreads) {
        const int i = x / TJ, jj = x % TJ;
        if (jj < jn) {
          double psi = 0.0;
          for (int a = 0; a < Ra; ++a) {
            const double* zr = Zn + ((int64_t)a * Kn + i) * Rb;
            const double* br = Bs + jj * ldB + a * Rb;
#pragma unroll 8
            for (int b = 0; b < Rb; ++b) psi += zr[b] * br[b];
          }
          const double d = Ls[i * ldL + jj] - psi;
          rsum += d * d;
        }
      }
    }
  }
  const int nout = nM + (g.gram_direct ? RR * RR : 0);
  double* out = g.part + (int64_t)blockIdx.x * (nout + 1);
  if (accum) {
    const int r16 = lane & 15, g4 = lane >> 4;
#pragma unroll
    for (int s = 0; s < kAcTiles; ++s) {
      const int q = wid + 16 * s;
      if (q < ntot) {
        const bool isM = q < ntM;
        const int qq = isM ? q : q - ntM;
        const int mt = qq / NT, nt = qq % NT;
        const int col = nt * 16 + r16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mt * 16 + 4 * r + g4;
          if (isM) {
            if (row < Kn && col < RR) out[row * RR + col] = acc[s][r];
          } else {
            if (row < RR && col < RR) out[nM + row * RR + col] = acc[s][r];
          }
        }
      }
    }
  }
  rsum = block_sum(rsum, red);
  if (tid == 0) out[nout] = rsum;
}

// ---------------------------------------------------------------------------------------
// C = A B on the FP64 matrix cores for an (Mp x Kp) by (Kp x Np) product, Mp and Np
// multiples of 16, Kp of 4; A(m, k) = A[m * lda + k * ska], B(k, n) = B[k * ldb + n],
// C row-major with ldc.  Output tiles are spread over the block's wavefronts.
__device__ void gemm_f64(const double* A, int lda, int ska, const double* B, int ldb, double* C,
                         int ldc, int Mp, int Np, int Kp) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int MT = Mp / 16, NT = Np / 16;
  for (int q = wid; q < MT * NT; q += nw) {
    const int mt = q / NT, nt = q % NT;
    f64x4 c = {0.0, 0.0, 0.0, 0.0};
    const double* ap = A + (mt * 16 + r16) * lda + g4 * ska;
    const double* bp = B + g4 * ldb + nt * 16 + r16;
    for (int k0 = 0; k0 < Kp; k0 += 4) c = mma_f64(ap[k0 * ska], bp[k0 * ldb], c);
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(mt * 16 + 4 * r + g4) * ldc + nt * 16 + r16] = c[r];
  }
}

// Gram of core n's least squares from transfer matrices (every core except n is read):
// sum_j S_j (x) S_j = E_{n+1} .. E_{n-1}.  xt: LDS workspace of 3 tdim^2 + 64 tdim + ztotal
// doubles (3 tdim^2 + 64 tdim when the cores are already in LDS at ``Zstaged``); G: RR x RR
// output (LDS or global).  Called by a whole work-group.
__device__ void transfer_gram(const double* __restrict__ Z, int64_t ztotal, int N, int n,
                              const int64_t* zoff, const int* Kc, const int* Rc, int tdim, int Ra,
                              int Rb, double* xt, double* G, const double* Zstaged) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int RR = Ra * Rb;
  // Gram from transfer matrices: sum_j S_j (x) S_j = E_{n+1} E_{n+2} ... E_{n-1},
  // E_m[(p,p'),(q,q')] = sum_i Z_m[p,i,q] Z_m[p',i,q']; entry [(b,b'),(a,a')] of the
  // product is Gram[(a,b),(a',b')].  Buffers are D x D (D = pad16(max R^2)), zero padded.
  const int D = tdim;
  double* Tm = xt;
  double* Em = Tm + D * D;
  double* Tn = Em + D * D;
  double* Fz = Tn + D * D;   // Kp x W slice matrix, Kp <= 64
  const double* Zs = Zstaged ? Zstaged : Fz + 64 * D;  // cores
  if (!Zstaged) {
    double* Zw = Fz + 64 * D;
    double zt[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      const int64_t x = tid + (int64_t)e * nth;
      zt[e] = x < ztotal ? Z[x] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      const int64_t x = tid + (int64_t)e * nth;
      if (x < ztotal) Zw[x] = zt[e];
    }
  }
  for (int x = tid; x < 3 * D * D; x += nth) Tm[x] = 0.0;
  __syncthreads();
  const int Rn1 = Rc[(n + 1) % N];
  for (int t = 1; t < N; ++t) {
    const int m = (n + t) % N;
    const int Rp = Rc[m], Rq = Rc[(m + 1) % N], Km = Kc[m];
    const int Kp = (Km + 3) / 4 * 4, W = pad16(Rp * Rq);
    const double* Zm = Zs + zoff[m];
    // Fz[i][(p,q)] = Z_m[p,i,q], zero padded
    for (int x = tid; x < Kp * W; x += nth) {
      const int i = x / W, c = x % W;
      const int p = c / Rq, q = c % Rq;
      Fz[x] = (i < Km && c < Rp * Rq) ? Zm[(p * Km + i) * Rq + q] : 0.0;
    }
    __syncthreads();
    // F = Fz^T Fz (W x W) into Tn, then scattered into the E layout
    gemm_f64(Fz, 1, W, Fz, W, Tn, D, W, W, Kp);
    __syncthreads();
    double* dst = (t == 1) ? Tm : Em;
    for (int x = tid; x < D * D; x += nth) {  // whole buffer: zero outside the block
      const int row = x / D, col = x % D;
      double v = 0.0;
      if (row < Rp * Rp && col < Rq * Rq) {
        const int p = row / Rp, pp = row % Rp, q = col / Rq, qq = col % Rq;
        v = Tn[(p * Rq + q) * D + pp * Rq + qq];
      }
      dst[x] = v;
    }
    __syncthreads();
    if (t > 1) {
      const int mp = pad16(Rn1 * Rn1), np = pad16(Rq * Rq);
      gemm_f64(Tm, D, 1, Em, D, Tn, D, mp, np, pad16(Rp * Rp));
      __syncthreads();
      for (int x = tid; x < D * D; x += nth) {
        const int row = x / D, col = x % D;
        Tm[x] = (row < mp && col < np) ? Tn[x] : 0.0;
      }
      __syncthreads();
    }
  }
  // Tm is R_{n+1}^2 x R_n^2
  const int Rb2 = Rb, Ra2 = Ra;
  for (int x = tid; x < RR * RR; x += nth) {
    const int r1 = x / RR, r2 = x % RR;
    const int a = r1 / Rb2, b = r1 % Rb2, a2 = r2 / Rb2, b2 = r2 % Rb2;
    G[x] = Tm[(b * Rb2 + b2) * D + (a * Ra2 + a2)];
  }
  __syncthreads();
}

template <int RMAX>
__global__ __launch_bounds__(kSolveThreads) void als_solve2_kernel(AlsSolveArgs g) {
  if (*g.done) return;
  extern __shared__ __align__(16) double sm[];
  const int RR = g.RR, Kn = g.Kn, nM = Kn * RR;
  double* M = sm;               // Kn x RR, overwritten by the new core rows
  double* G = sm + nM;          // RR x RR, lower Cholesky factor in place
  double* invd = G + RR * RR;   // RR
  double* cvec = invd + RR;     // 64
  double* xt = cvec + 64 + 1024;  // transfer-matrix workspace
  __shared__ double red[16];
  __shared__ int failed;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nstore = nM + (g.gram_direct ? RR * RR : 0);  // partial record length (+1)
  if (g.report_sweep >= 0) {
    double s = 0.0;
    for (int c = tid; c < g.nparts; c += nth) s += g.part[(int64_t)c * (nstore + 1) + nstore];
    s = block_sum(s, red);
    if (tid == 0) {
      const double e = sqrt(s / g.pn2[0]);
      const int sw = g.report_sweep;
      g.trace[sw] = e;
      *g.sweeps_run = sw + 1;
      if (g.tol > 0.0 && sw >= 1 && fabs(e - g.trace[sw - 1]) < g.tol) *g.done = 1;
    }
    __syncthreads();
    if (*g.done || g.report_only) return;
  }
  for (int o = tid; o < nstore; o += nth) sm[o] = g.red[o];  // the summed records
  if (tid == 0) failed = 0;
  if (g.gram_in) {
    for (int x = tid; x < RR * RR; x += nth) G[x] = g.gram_in[x];
  } else if (!g.gram_direct) {
    transfer_gram(g.Z, g.ztotal, g.N, g.n, g.zoff, g.Kc, g.Rc, g.tdim, g.Ra, g.Rb, xt, G);
  }
  __syncthreads();
  if constexpr (RMAX > 0) {
    // RMAX here is the number of augmented-matrix elements per thread; the solution entry
    // (r = a R_{n+1} + b, i) is core entry (a, i, b), written straight to the core
    double* rowbuf = cvec + 64;     // 2 x 256
    double* colbuf = rowbuf + 512;  // 2 x 256
    double* Zn = g.Zn;
    const int Rb = g.Rb;
    auto store = [=](int r, int i, double v) {
      Zn[((int64_t)(r / Rb) * Kn + i) * Rb + (r % Rb)] = v;
    };
    if (!gauss_jordan<RMAX>(G, M, store, rowbuf, colbuf, RR, Kn, &failed)) {
      if (tid == 0) atomicOr(g.status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
      return;
    }
    return;
  } else {
    for (int j = 0; j < RR; ++j) {
      if (tid == 0) {
        const double d = G[j * RR + j];
        if (!(d > 0.0))
          failed = 1;
        else
          G[j * RR + j] = sqrt(d);
      }
      __syncthreads();
      if (failed) break;
      const double ljj = G[j * RR + j];
      for (int i = j + 1 + tid; i < RR; i += nth) G[i * RR + j] /= ljj;
      __syncthreads();
      const int rem = RR - j - 1;
      for (int x = tid; x < rem * rem; x += nth) {
        const int i = j + 1 + x / rem, k = j + 1 + x % rem;
        if (k <= i) G[i * RR + k] -= G[i * RR + j] * G[k * RR + j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (failed) {
      if (tid == 0) atomicOr(g.status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
      return;
    }
    for (int r = tid; r < RR; r += nth) invd[r] = 1.0 / G[r * RR + r];
    __syncthreads();
    for (int row = tid; row < Kn; row += nth) {
      double* m = M + (int64_t)row * RR;
      for (int r = 0; r < RR; ++r) {
        double sacc = 0.0;
        for (int k = 0; k < r; ++k) sacc += G[r * RR + k] * m[k];
        m[r] = (m[r] - sacc) * invd[r];
      }
      for (int r = RR - 1; r >= 0; --r) {
        double sacc = 0.0;
        for (int k = r + 1; k < RR; ++k) sacc += G[k * RR + r] * m[k];
        m[r] = (m[r] - sacc) * invd[r];
      }
    }
    __syncthreads();
    for (int x = tid; x < nM; x += nth) {
      const int i = x / RR, r = x % RR;
      const int a = r / g.Rb, b = r % g.Rb;
      g.Zn[((int64_t)a * Kn + i) * g.Rb + b] = M[x];
    }
  }
}

// The accumulation's records summed element by element in a fixed order (one thread per
// element, batches of 32 loads issued together; the last batch reads clamped valid records
// and masks them by a multiply, so no record is fetched by a lone dependent load).
__global__ __launch_bounds__(256) void als_reduce_kernel(const double* __restrict__ part,
                                                         int nparts, int nstore,
                                                         double* __restrict__ red) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= nstore) return;
  const double* src = part + o;
  const int64_t st = nstore + 1;
  const int last = nparts - 1;
  double s = 0.0;
  for (int c = 0; c < nparts; c += 32) {
    double v[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      const int cc = c + e <= last ? c + e : last;
      v[e] = src[(int64_t)cc * st] * (c + e <= last ? 1.0 : 0.0);
    }
    __builtin_amdgcn_sched_barrier(0);  // all 32 loads ahead of the sums
#pragma unroll
    for (int e = 0; e < 32; ++e) s += v[e];
  }
  red[o] = s;
}

// The update's solve by the blocked Gauss-Jordan of ps_solve (NW wavefronts, TPW tiles each; the
// matrix cores, not the wavefront count, bound the elimination), M and the Gram read straight
// from the summed records (or the Gram from the accumulation launch).
constexpr int kSolveW = 256;
template <int NW, int TPW>
__global__ __launch_bounds__(NW * 64) void als_solve_mfma_kernel(AlsSolveArgs g) {
  if (*g.done) return;
  extern __shared__ __align__(16) double sm[];
  __shared__ double red16[16];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int RR = g.RR, Kn = g.Kn, nM = Kn * RR;
  if (g.report_sweep >= 0) {
    const int nstore = nM + (g.gram_direct ? RR * RR : 0);
    double s = 0.0;
    for (int c = tid; c < g.nparts; c += nth) s += g.part[(int64_t)c * (nstore + 1) + nstore];
    s = block_sum(s, red16);
    if (tid == 0) {
      const double e = sqrt(s / g.pn2[0]);
      const int sw = g.report_sweep;
      g.trace[sw] = e;
      *g.sweeps_run = sw + 1;
      if (g.tol > 0.0 && sw >= 1 && fabs(e - g.trace[sw - 1]) < g.tol) *g.done = 1;
    }
    __syncthreads();
    if (*g.done || g.report_only) return;
  }
  const double* Gp = g.gram_in ? g.gram_in : g.red + nM;
  for (int kc0 = 0; kc0 < Kn; kc0 += g.kwin) {  // right-hand sides in windows of kwin columns
    const int kcols = Kn - kc0 < g.kwin ? Kn - kc0 : g.kwin;
    if (!ps_solve<NW, TPW, kSolveW>(g.red, Gp, RR, Kn, kc0, kcols, g.Rb, g.Zn, sm,
                                    sm + 2 * 4 * kSolveW, [] {})) {
      if (tid == 0) atomicOr(g.status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
      return;
    }
  }
}

// The variant of als_solve_mfma_kernel for a shape: 8 wavefronts (two per SIMD, so each holds
// up to 12 tiles in registers) with 1, 2, 4, 8 or 12 tiles each, and the right-hand-side window
// ``kwin`` (all of K'_n when the augmented matrix fits 96 tiles, else the widest window that
// does); nullptr if not even one column fits.
static const void* solve_mfma_fn(int RR, int Kn, int* threads, int* kwin) {
  const int RR4 = (RR + 3) & ~3, MT = (RR4 + 15) / 16;
  int win = Kn;
  const int ntmax = 96 / MT;  // tile columns that fit beside MT tile rows
  if (((RR4 + win + 15) / 16) > ntmax) win = ntmax * 16 - RR4;
  if (win < 1 || RR4 + win > kSolveW) return nullptr;
  *kwin = win;
  const int tiles = MT * ((RR4 + win + 15) / 16);
  *threads = 512;
  if (tiles <= 8) return (const void*)als_solve_mfma_kernel<8, 1>;
  if (tiles <= 16) return (const void*)als_solve_mfma_kernel<8, 2>;
  if (tiles <= 32) return (const void*)als_solve_mfma_kernel<8, 4>;
  if (tiles <= 64) return (const void*)als_solve_mfma_kernel<8, 8>;
  if (tiles <= 96) return (const void*)als_solve_mfma_kernel<8, 12>;
  return nullptr;
}

// ---------------------------------------------------------------------------------------
static int64_t accum_words(int Kn, int RR, int64_t ztotal, int tj) {
  const int64_t z = ztotal <= kZldsMax ? zwords(ztotal) : 0;
  return z + (int64_t)tj * (pad16(RR) + 1) + (int64_t)pad16(Kn) * (tj + 1);
}

static int accum_tj(int Kn, int RR, int64_t ztotal) {
  for (int tj = 128; tj >= 32; tj /= 2)
    if (accum_words(Kn, RR, ztotal, tj) * 8 <= 150 * 1024) return tj;
  return 0;
}

static size_t solve_lds(int Kn, int RR, int gram_direct, int tdim, int64_t ztotal) {
  int64_t w = (int64_t)Kn * RR + (int64_t)RR * RR + RR + 64 + 1024;  // + row/column buffers
  // the transfer-matrix workspace (the Gauss-Jordan solution goes straight to the core)
  const int64_t xt = gram_direct ? 0 : 3 * (int64_t)tdim * tdim + 64 * (int64_t)tdim + ztotal;
  return (size_t)(w + xt) * 8;
}

int als2_tdim(int rmax) { return pad16(rmax * rmax); }

bool als2_supported(int Kn, int RR, int64_t J, int64_t ztotal, int gram_direct, int tdim,
                    int maxK) {
  const int tj = accum_tj(Kn, RR, ztotal);
  const int NT = pad16(RR) / 16, MT = pad16(Kn) / 16;
  const int tiles = MT * NT + (gram_direct ? NT * NT : 0);
  int thr = 0, kwin = 0;
  const bool mfma_solve = solve_mfma_fn(RR, Kn, &thr, &kwin) != nullptr;
  // the transfer-matrix Gram is formed by an extra work-group of the accumulation launch
  const bool gram_fits =
      gram_direct || (3 * (int64_t)tdim * tdim + 64 * (int64_t)tdim + ztotal) * 8 <= 150 * 1024;
  return tj > 0 && Kn <= 256 && J < (1LL << 31) && tiles <= 16 * kAcTilesMax && gram_fits &&
         (mfma_solve || solve_lds(Kn, RR, gram_direct, tdim, ztotal) <= 150 * 1024) &&
         (gram_direct || (ztotal <= 12 * 512 && maxK <= 64));
}

// Number of partial records the accumulation writes (its grid).
int64_t als2_parts(int Kn, int RR, int64_t J, int64_t ztotal) {
  const int tj = accum_tj(Kn, RR, ztotal);
  if (tj == 0) return 0;  // shape not taken by this path
  const int64_t ntiles = (J + tj - 1) / tj;
  const int64_t grid = ntiles < 64 ? ntiles : 64;
  const int64_t per = (ntiles + grid - 1) / grid;
  return (ntiles + per - 1) / per;
}

template <int TJ, int NTW>
static const void* accum_fn(int rmax) {
  if (rmax <= 4) return (const void*)als_accum_kernel<4, TJ, NTW>;
  if (rmax <= 8) return (const void*)als_accum_kernel<8, TJ, NTW>;
  if (rmax <= 16) return (const void*)als_accum_kernel<16, TJ, NTW>;
  return (const void*)als_accum_kernel<RTR_MAX_RANK, TJ, NTW>;
}

template <int TJ>
static const void* accum_pick(int rmax, int ntw) {
  if (ntw <= 1) return accum_fn<TJ, 1>(rmax);
  if (ntw <= 2) return accum_fn<TJ, 2>(rmax);
  return accum_fn<TJ, kAcTilesMax>(rmax);
}

hipError_t launch_als_accum(AlsArgs2 g, int rmax, hipStream_t s) {
  const int tj = accum_tj(g.Kn, g.RR, g.ztotal);
  const int64_t ntiles = (g.J + tj - 1) / tj;
  const int64_t grid = als2_parts(g.Kn, g.RR, g.J, g.ztotal);
  g.tiles_per_wg = (ntiles + grid - 1) / grid;
  g.zlds = g.ztotal <= kZldsMax;
  size_t lds = (size_t)accum_words(g.Kn, g.RR, g.ztotal, tj) * 8;
  if (g.gram_extra)
    lds = std::max(lds, (size_t)(3 * (int64_t)g.tdim * g.tdim + 64 * (int64_t)g.tdim + g.ztotal) * 8);
  const int NT = pad16(g.RR) / 16, MT = pad16(g.Kn) / 16;
  const int ntot = MT * NT + (g.gram_direct ? NT * NT : 0);
  const int ntw = (ntot + 15) / 16;  // output tiles per wavefront
  const void* fn = tj == 128 ? accum_pick<128>(rmax, ntw)
                 : tj == 64  ? accum_pick<64>(rmax, ntw)
                             : accum_pick<32>(rmax, ntw);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("als_accum", s);
  void* args[] = {&g};
  e = hipLaunchKernel(fn, dim3((unsigned)(grid + (g.gram_extra ? 1 : 0))), dim3(kAcThreads), args,
                      lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_als_solve2(AlsSolveArgs g, hipStream_t s) {
  hipError_t e;
  if (!g.report_only) {  // the records summed once, by many work-groups
    const int nstore = g.Kn * g.RR + (g.gram_direct ? g.RR * g.RR : 0);
    prof_begin("als_reduce", s);
    hipLaunchKernelGGL(als_reduce_kernel, dim3((unsigned)((nstore + 255) / 256)), dim3(256), 0, s,
                       g.part, g.nparts, nstore, g.red);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int threads = 0;
  const void* mf = solve_mfma_fn(g.RR, g.Kn, &threads, &g.kwin);
  if (mf && (g.gram_in || g.gram_direct || g.report_only)) {
    const size_t lds = (size_t)(2 * 4 * kSolveW + 2 * kSolveW * 4) * sizeof(double);
    if ((e = hipFuncSetAttribute(mf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
      return e;
    prof_begin("als_solve", s);
    void* args[] = {&g};
    e = hipLaunchKernel(mf, dim3(1), dim3((unsigned)threads), args, lds, s);
    prof_end(s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  const size_t lds = solve_lds(g.Kn, g.RR, g.gram_direct, g.tdim, g.ztotal);
  // Gauss-Jordan path: augmented rows of at most 256 entries (the LDS row/column buffers),
  // elements spread over kSolveThreads threads
  const int ne = (g.RR + g.Kn <= 256) ? g.RR * (g.RR + g.Kn) : (1 << 30);
  const int T = kSolveThreads;
  const void* fn = ne <= T ? (const void*)als_solve2_kernel<1>
                 : ne <= 2 * T ? (const void*)als_solve2_kernel<2>
                 : ne <= 4 * T ? (const void*)als_solve2_kernel<4>
                 : ne <= 8 * T ? (const void*)als_solve2_kernel<8>
                 : ne <= 16 * T ? (const void*)als_solve2_kernel<16>
                                : (const void*)als_solve2_kernel<0>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("als_solve", s);
  void* args[] = {&g};
  e = hipLaunchKernel(fn, dim3(1), dim3(kSolveThreads), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// TR-ALS in one cooperative launch: every sweep and core update of one decomposition.
//
// Each work-group keeps all cores in LDS.  Per core update n, with the columns j of P_<n>
// cut into tiles of TJ (tile t on work-group t mod G):
//   A  each work-group forms the subchain rows B of its tiles from the LDS cores and
//      accumulates M = P_<n> B and the Gram B^T B on the FP64 matrix cores into its record
//      in ``part``; on the first update of a sweep it also accumulates the residual
//      ||P - Psi(Z)||^2 of its columns with the cores of the sweep before (Psi tile = Z_n B^T,
//      also on the matrix cores)
//   -- grid barrier --
//   B  the records are summed in a fixed order, the elements split over the work-groups
//   -- grid barrier --
//   C  every work-group reads the summed M and Gram and solves the normal equations by
//      Gauss-Jordan itself (4x4 pivot blocks, the eliminations on the FP64 matrix cores); the
//      arithmetic is identical in each, so all LDS copies of core n receive the same values
//      and no third barrier is needed.
// The P tile of the next update is loaded into registers during the solve (issued after the
// solve's own loads), so its latency overlaps the elimination.  A grid barrier is an agent-scope release/acquire on a monotonic
// arrival counter (zero at launch); its wait is bounded: a barrier that does not complete
// sets RTR_STATUS_SYNC_TIMEOUT and every work-group leaves the launch.
constexpr int kPsThreads = 512;  // 8 wavefronts
constexpr int kPsTiles = 4;      // 16x16 FP64 output tiles per wavefront (M and Gram)
constexpr int kPsSolveW = 128;   // bound of the solve's augmented width RR4 + K'_n

__device__ __forceinline__ bool ps_grid_sync(unsigned* bar, unsigned nblk, unsigned& epoch,
                                             unsigned limit, unsigned* status, int* s_fail) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have reached the L2
  __syncthreads();
  if (threadIdx.x == 0 && !*s_fail) {
    // release: the XCD's L2 written back, then the arrival; the wait polls with relaxed
    // loads (no cache maintenance per poll) and acquires once, invalidating stale lines
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    ++epoch;
    const unsigned target = epoch * nblk;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > limit) {
        *s_fail = 1;
        atomicOr(status, (unsigned)RTR_STATUS_SYNC_TIMEOUT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return *s_fail == 0;
}

// Output tile qq of the accumulation: M tiles (mt, nt) first, then the Gram's upper
// block-triangle (nt >= mt) row by row.
__device__ __forceinline__ void ps_tile(int qq, int ntM, int NT, int& mt, int& nt) {
  if (qq < ntM) {
    mt = qq / NT;
    nt = qq % NT;
    return;
  }
  int q2 = qq - ntM, row = 0;
  while (q2 >= NT - row) {
    q2 -= NT - row;
    ++row;
  }
  mt = row;
  nt = row + q2;
}

// Geometry of core update n (the cyclic order after n, and the subchain's cores).
struct PsGeom {
  int Kn, Ra, Rb, RR, nM, J, ntiles, strideN;
  int cycK[7], chI[7], chRb[7];
  int cycStride[7], chOff[7];
  int zoffN;
};

__device__ __forceinline__ PsGeom ps_geom(const AlsPersistArgs& g, int n, int TJ) {
  PsGeom q;
  const int N = g.N;
  q.Kn = g.K[n];
  q.Ra = g.R[n];
  q.Rb = g.R[(n + 1) % N];
  q.RR = q.Ra * q.Rb;
  q.nM = q.Kn * q.RR;
  q.J = (int)(g.total / q.Kn);
  q.ntiles = (q.J + TJ - 1) / TJ;
  q.strideN = (int)g.strideP[n];
  q.zoffN = (int)g.zoff[n];
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int m = (n + 1 + t) % N;
    q.cycK[t] = g.K[m];
    q.cycStride[t] = (int)g.strideP[m];
    q.chI[t] = g.K[m];
    q.chRb[t] = g.R[(m + 1) % N];
    q.chOff[t] = (int)g.zoff[m];
  }
  return q;
}

// P_<n>[:, tile t] into registers: element x = tid + e * kPsThreads is (i, jj) = (x / TJ, x % TJ),
// KPER * kPsThreads >= K'_n TJ.
template <int TJ, int KPER>
__device__ __forceinline__ void ps_load_p(const AlsPersistArgs& g, const PsGeom& q, int t,
                                          double (&pv)[KPER]) {
  static_assert(kPsThreads % TJ == 0, "a thread's elements share one column of the tile");
  const int tid = threadIdx.x, N = g.N;
  const int j0 = t * TJ, jn = min(TJ, q.J - j0);
  const int jj = tid % TJ, i0 = tid / TJ;
  constexpr int kRows = kPsThreads / TJ;  // rows between a thread's elements
  const bool col_ok = t < q.ntiles && jj < jn;
  int base = 0;
  if (col_ok) {
    int rem = j0 + jj;
#pragma unroll
    for (int u = 6; u >= 0; --u) {
      if (u <= N - 2) {
        const int d = q.cycK[u];
        const int qq = rem / d;
        base += (rem - qq * d) * q.cycStride[u];
        rem = qq;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < KPER; ++e) {
    const int i = i0 + kRows * e;
    pv[e] = (col_ok && i < q.Kn) ? g.P[base + i * q.strideN] : 0.0;
  }
}

// Inverse of a 4x4 pivot block by the 2x2 block formula (Schur complement of the leading 2x2
// block; two divisions), row-major into ``out``.  Returns false unless the leading 2x2 block
// and its Schur complement are positive definite (for a symmetric block: unless the block is).
__device__ __forceinline__ bool ps_inv4(const double* p, int ld, double out[16]) {
  const double a00 = p[0], a01 = p[1], a10 = p[ld], a11 = p[ld + 1];
  const double b00 = p[2], b01 = p[3], b10 = p[ld + 2], b11 = p[ld + 3];
  const double c00 = p[2 * ld], c01 = p[2 * ld + 1], c10 = p[3 * ld], c11 = p[3 * ld + 1];
  const double d00 = p[2 * ld + 2], d01 = p[2 * ld + 3], d10 = p[3 * ld + 2], d11 = p[3 * ld + 3];
  const double da = a00 * a11 - a01 * a10;
  if (!(a00 > 0.0) || !(da > 0.0)) return false;
  const double ia = 1.0 / da;
  const double i00 = a11 * ia, i01 = -a01 * ia, i10 = -a10 * ia, i11 = a00 * ia;
  // E = A^-1 B, F = C A^-1, S = D - C E
  const double e00 = i00 * b00 + i01 * b10, e01 = i00 * b01 + i01 * b11;
  const double e10 = i10 * b00 + i11 * b10, e11 = i10 * b01 + i11 * b11;
  const double f00 = c00 * i00 + c01 * i10, f01 = c00 * i01 + c01 * i11;
  const double f10 = c10 * i00 + c11 * i10, f11 = c10 * i01 + c11 * i11;
  const double s00 = d00 - (c00 * e00 + c01 * e10), s01 = d01 - (c00 * e01 + c01 * e11);
  const double s10 = d10 - (c10 * e00 + c11 * e10), s11 = d11 - (c10 * e01 + c11 * e11);
  const double ds = s00 * s11 - s01 * s10;
  if (!(s00 > 0.0) || !(ds > 0.0)) return false;
  const double is = 1.0 / ds;
  const double t00 = s11 * is, t01 = -s01 * is, t10 = -s10 * is, t11 = s00 * is;  // S^-1
  // inverse = [A^-1 + E S^-1 F, -E S^-1; -S^-1 F, S^-1]
  const double g00 = e00 * t00 + e01 * t10, g01 = e00 * t01 + e01 * t11;  // E S^-1
  const double g10 = e10 * t00 + e11 * t10, g11 = e10 * t01 + e11 * t11;
  out[0] = i00 + g00 * f00 + g01 * f10;
  out[1] = i01 + g00 * f01 + g01 * f11;
  out[2] = -g00;
  out[3] = -g01;
  out[4] = i10 + g10 * f00 + g11 * f10;
  out[5] = i11 + g10 * f01 + g11 * f11;
  out[6] = -g10;
  out[7] = -g11;
  out[8] = -(t00 * f00 + t01 * f10);
  out[9] = -(t00 * f01 + t01 * f11);
  out[10] = t00;
  out[11] = t01;
  out[12] = -(t10 * f00 + t11 * f10);
  out[13] = -(t10 * f01 + t11 * f11);
  out[14] = t10;
  out[15] = t11;
  return true;
}

// Gauss-Jordan elimination on [Gram | M^T] without pivoting (the Gram is symmetric positive
// definite: every pivot block is a Schur complement of it, itself positive definite), four
// pivots per step, on the FP64 matrix cores, by a work-group of NW wavefronts.  Mp is M
// (K'_n x RR row-major), Gp the Gram (RR x RR); the right-hand sides taken are the columns
// kc0 .. kc0 + kcols - 1 of M^T (the solve may run in windows of them, each eliminating the
// Gram anew); SW bounds the augmented width RR4 + kcols and sizes the
// LDS buffers (rowbuf 2 x 4 x SW, colbuf 2 x SW x 4 doubles).  The RR4 x W4 augmented matrix
// (RR rounded up to a multiple of 4, the extra unknowns decoupled by an identity block;
// W4 = RR4 + K'_n) lives in 16x16 accumulator tiles: tile q = wid + NW u of the MT x NT grid,
// the lane holding rows 4i + (lane / 16) and column lane % 16 of it.  Step k (pivots
// k..k+3): the owners publish the pivot rows and columns (double-buffered LDS); barrier;
// wavefront 0 alone inverts the 4x4 pivot block P and overwrites the published pivot rows with
// R = P^-1 C[pivot rows, :]; barrier; then every tile takes one 16x16x4 product,
//   C <- C - A R,   A = C[:, pivot columns] with the pivot rows zeroed,
// after which the pivot rows are set to R.  Writing R in place, rather than forming it as
// C_p - (P - I) R, keeps the pivot rows free of a cancellation whose error grows with the size
// of P's entries; inverting in one wavefront keeps the others off the FP64 units while the
// chain of dependent operations runs.  ``prefetch`` runs once the tiles' loads are issued
// (loads it issues stay in flight during the elimination).  The solution columns are written
// into core n (Zn).  Returns false, leaving the core unchanged, if a pivot block is not
// positive definite.
template <int NW, int TPW, int SW, class Prefetch>
__device__ bool ps_solve(const double* Mp, const double* Gp, int RR, int Kn, int kc0, int kcols,
                         int Rb, double* Zn, double* rowbuf, double* colbuf, Prefetch&& prefetch) {
  const int RR4 = (RR + 3) & ~3, W4 = RR4 + kcols;
  const int MT = (RR4 + 15) / 16, NT = (W4 + 15) / 16;
  // the wavefront index in a scalar register: the tile indices and their LDS offsets derived
  // from it then stay scalar instead of occupying vector registers per tile
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, g4 = lane >> 4;
  f64x4 c[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int q = wid + NW * u;
    const int mt = q / NT, nt = q % NT;
    const int col = nt * 16 + r16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = mt * 16 + 4 * i + g4;
      double v = 0.0;
      if (q < MT * NT) {
        if (col < RR4)
          v = (row < RR && col < RR) ? Gp[row * RR + col] : (row == col ? 1.0 : 0.0);
        else if (col < W4 && row < RR)
          v = Mp[(kc0 + col - RR4) * RR + row];
      }
      c[u][i] = v;
    }
  }
  prefetch();
  __shared__ int s_ok;
  bool ok = true;
  for (int k = 0, par = 0; k < RR4; k += 4, par ^= 1) {
    double* rb = rowbuf + par * 4 * SW;  // pivot rows [4][W4]
    double* cb = colbuf + par * SW * 4;         // pivot columns [RR4][4]
    const int mp = k >> 4, ip = (k & 15) >> 2, np = k >> 4, cp = k & 15;
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int q = wid + NW * u;
      if (q < MT * NT) {
        const int mt = q / NT, nt = q % NT;
        if (mt == mp) {
          const double x = ip == 0 ? c[u][0] : ip == 1 ? c[u][1] : ip == 2 ? c[u][2] : c[u][3];
          rb[g4 * SW + nt * 16 + r16] = x;
        }
        if (nt == np && r16 >= cp && r16 < cp + 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i) cb[(mt * 16 + 4 * i + g4) * 4 + (r16 - cp)] = c[u][i];
        }
      }
    }
    __syncthreads();
    if (wid == 0) {
      double pin[16] = {};
      const bool good = ps_inv4(rb + k, SW, pin);
      // each lane rewrites its own columns only, after reading them (the pivot block itself
      // was read above), so the in-place update needs no further synchronisation
      for (int col = lane; col < NT * 16; col += 64) {
        double x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = rb[m * SW + col];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          rb[g * SW + col] = pin[4 * g] * x[0] + pin[4 * g + 1] * x[1] + pin[4 * g + 2] * x[2] +
                             pin[4 * g + 3] * x[3];
      }
      if (lane == 0) s_ok = good ? 1 : 0;
    }
    __syncthreads();
    ok = s_ok != 0;
    if (!ok) break;  // the same outcome in every lane
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
      const int q = wid + NW * u;
      if (q < MT * NT) {
        const int mt = q / NT, nt = q % NT;
        const int col = nt * 16 + r16, row = mt * 16 + r16;
        const double b = rb[g4 * SW + col];
        const double a = (row >= k && row < k + 4) ? 0.0 : cb[row * 4 + g4];
        c[u] = mma_f64(-a, b, c[u]);
        if (mt == mp) {  // the pivot rows become R (this lane's B operand)
          if (ip == 0) c[u][0] = b;
          if (ip == 1) c[u][1] = b;
          if (ip == 2) c[u][2] = b;
          if (ip == 3) c[u][3] = b;
        }
      }
    }
  }
  __syncthreads();
  if (!ok) return false;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int q = wid + NW * u;
    if (q < MT * NT) {
      const int mt = q / NT, nt = q % NT;
      const int col = nt * 16 + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = mt * 16 + 4 * i + g4;
        if (row < RR && col >= RR4 && col < W4)
          Zn[((row / Rb) * Kn + kc0 + (col - RR4)) * Rb + (row % Rb)] = c[u][i];
      }
    }
  }
  return true;
}

// Tiles per wavefront of ps_solve (1, 2 or 4; 0 if the augmented matrix exceeds 32 tiles).
static __host__ __device__ inline int ps_tpw(int RR, int Kn) {
  const int RR4 = (RR + 3) & ~3, W4 = RR4 + Kn;
  const int tiles = ((RR4 + 15) / 16) * ((W4 + 15) / 16);
  if (W4 > kPsSolveW) return 0;
  return tiles <= 8 ? 1 : tiles <= 16 ? 2 : tiles <= 32 ? 4 : 0;
}

// RM: rank bound of the subchain registers; TPW: tiles per wavefront of the solve; TJ: tile
// width; KT: bound of K'_n (sizes the register tile of P).
template <int RM, int TPW, int TJ, int KT>
__global__ __launch_bounds__(kPsThreads) void als_persist_kernel(AlsPersistArgs g) {
  extern __shared__ __align__(16) double sm[];
  __shared__ double wred[16];
  __shared__ int s_fail;
  constexpr int KPER = (KT * TJ + kPsThreads - 1) / kPsThreads;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int N = g.N, G = g.G;
  const unsigned nblk = (unsigned)G;
  double* Zs = sm;
  double* U = sm + zwords(g.ztotal);
  for (int x = tid; x < (int)g.ztotal; x += kPsThreads) Zs[x] = g.Z[x];
  // the tile buffers start at zero: rows of B beyond a partial tile are rewritten as zeros by
  // every build, and padding rows and columns only feed outputs that are discarded
  for (int x = tid; x < (int)g.ubuf; x += kPsThreads) U[x] = 0.0;
  if (tid == 0) s_fail = 0;
  const double pn2 = g.pn2[0];
  unsigned epoch = 0;
  double eprev = 0.0;
  bool stop = false;
  const int S = g.max_sweeps;
  double pv[KPER];
  {
    const PsGeom q0 = ps_geom(g, 0, TJ);
    ps_load_p<TJ, KPER>(g, q0, blockIdx.x, pv);
  }
  __syncthreads();
  for (int s = 0; s <= S && !stop; ++s) {
    for (int n = 0; n < N; ++n) {
      const bool last = s == S;  // the closing pass: the residual of the final sweep only
      if (last && n > 0) break;
      const bool report = n == 0 && s > 0;
      const PsGeom q = ps_geom(g, n, TJ);
      const int Kn = q.Kn, Ra = q.Ra, Rb = q.Rb, RR = q.RR, nM = q.nM;
      const int nrec = q.ntiles < G ? q.ntiles : G;
      const int NT = pad16(RR) / 16, MT = pad16(Kn) / 16;
      const int ntM = MT * NT, ntot = ntM + NT * (NT + 1) / 2;
      const int ldB = pad16(RR) + 1, ldL = TJ + 1;
      const int rec_g = nM;            // Gram offset in a record
      const int rec_r = nM + RR * RR;  // residual slot
      // ---- A ---------------------------------------------------------------------------
      if ((int)blockIdx.x < nrec) {
        double* Bs = U;                  // [TJ][ldB], columns >= RR stay zero
        double* Ls = Bs + TJ * ldB;      // [pad16(Kn)][ldL]
        double* Zr = Ls + pad16(Kn) * ldL;  // core n as [pad16(Kn)][ldB] (rows i, cols (a,b))
        if (report)
          for (int x = tid; x < pad16(Kn) * ldB; x += kPsThreads) {
            const int i = x / ldB, r = x % ldB;
            double v = 0.0;
            if (i < Kn && r < RR) v = Zs[q.zoffN + ((r / Rb) * Kn + i) * Rb + (r % Rb)];
            Zr[x] = v;
          }
        f64x4 acc[kPsTiles];
#pragma unroll
        for (int u = 0; u < kPsTiles; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
        double rsum = 0.0;
        for (int t = blockIdx.x; t < q.ntiles; t += G) {
          const int j0 = t * TJ, jn = min(TJ, q.J - j0);
          __syncthreads();
          if (t != (int)blockIdx.x) ps_load_p<TJ, KPER>(g, q, t, pv);
#pragma unroll
          for (int e = 0; e < KPER; ++e) {
            const int x = tid + e * kPsThreads;
            const int i = x / TJ, jj = x % TJ;
            if (i < MT * 16) Ls[i * ldL + jj] = pv[e];
          }
          for (int x = KT * TJ + tid; x < MT * 16 * TJ; x += kPsThreads)  // rows KT.. (none)
            Ls[(x / TJ) * ldL + x % TJ] = 0.0;
          // subchain rows: item (jl, b) forms row b of S_j; every load is in range (clamped
          // indices, zero weights beyond the ranks), so the loads issue without branches
          for (int x = tid; x < TJ * Rb; x += kPsThreads) {
            const int jl = x / Rb, b = x % Rb;
            double v[RM], w[RM];
            int rem = j0 + (jl < jn ? jl : 0);
            int idx[7];
#pragma unroll
            for (int u = 6; u >= 0; --u) {
              if (u <= N - 2) {
                idx[u] = rem % q.chI[u];
                rem /= q.chI[u];
              }
            }
            {
              const int cR = q.chRb[0];
              const double* G0 = Zs + q.chOff[0] + (b * q.chI[0] + idx[0]) * cR;
#pragma unroll
              for (int c = 0; c < RM; ++c) {
                const double t0 = G0[c < cR ? c : cR - 1];
                v[c] = c < cR ? t0 : 0.0;
              }
            }
            int cur = q.chRb[0];
#pragma unroll
            for (int u = 1; u < 7; ++u) {
              if (u < N - 1) {
                const int cR = q.chRb[u];
                const int rs = q.chI[u] * cR;
                const double* Gm = Zs + q.chOff[u] + idx[u] * cR;
#pragma unroll
                for (int c = 0; c < RM; ++c) w[c] = 0.0;
#pragma unroll
                for (int a = 0; a < RM; ++a) {
                  const double* gr = Gm + (a < cur ? a : cur - 1) * rs;
#pragma unroll
                  for (int c = 0; c < RM; ++c) w[c] = fma(v[a], gr[c < cR ? c : cR - 1], w[c]);
                }
#pragma unroll
                for (int c = 0; c < RM; ++c) v[c] = c < cR ? w[c] : 0.0;
                cur = cR;
              }
            }
#pragma unroll
            for (int a = 0; a < RM; ++a)
              if (a < Ra) Bs[jl * ldB + a * Rb + b] = jl < jn ? v[a] : 0.0;
          }
          __syncthreads();
          if (!last) {  // M += P tile B tile, Gram += B tile^T B tile (FP64 matrix cores)
#pragma unroll
            for (int u = 0; u < kPsTiles; ++u) {
              const int qq = wid + 8 * u;
              if (qq < ntot) {
                const bool isM = qq < ntM;
                int mt, nt;
                ps_tile(qq, ntM, NT, mt, nt);
                const double* ap = isM ? Ls + (mt * 16 + r16) * ldL + g4
                                       : Bs + g4 * ldB + mt * 16 + r16;
                const int ast = isM ? 1 : ldB;
                const double* bp = Bs + g4 * ldB + nt * 16 + r16;
                f64x4 c = acc[u];
#pragma unroll 8
                for (int k0 = 0; k0 < TJ; k0 += 4) c = mma_f64(ap[k0 * ast], bp[k0 * ldB], c);
                acc[u] = c;
              }
            }
          }
          if (report) {  // (P - Z_n B^T)^2 over this tile; Psi tile on the matrix cores
            const int JT = TJ / 16;
            for (int qq = wid; qq < MT * JT; qq += 8) {
              const int mt = qq / JT, jt = qq % JT;
              const double* ap = Zr + (mt * 16 + r16) * ldB + g4;
              const double* bp = Bs + (jt * 16 + r16) * ldB + g4;
              f64x4 c = {0.0, 0.0, 0.0, 0.0};
              for (int k0 = 0; k0 < pad16(RR); k0 += 4) c = mma_f64(ap[k0], bp[k0], c);
              const int col = jt * 16 + r16;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = mt * 16 + 4 * r + g4;
                if (row < Kn && col < jn) {
                  const double d = Ls[row * ldL + col] - c[r];
                  rsum = fma(d, d, rsum);
                }
              }
            }
          }
        }
        double* out = g.part + (int64_t)blockIdx.x * g.rec;
#pragma unroll
        for (int u = 0; u < kPsTiles; ++u) {
          const int qq = wid + 8 * u;
          if (qq < ntot) {
            const bool isM = qq < ntM;
            int mt, nt;
            ps_tile(qq, ntM, NT, mt, nt);
            const int col = nt * 16 + r16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = mt * 16 + 4 * r + g4;
              if (isM) {
                if (row < Kn && col < RR) out[row * RR + col] = acc[u][r];
              } else if (row < RR && col < RR) {
                out[rec_g + row * RR + col] = acc[u][r];
                if (nt != mt) out[rec_g + col * RR + row] = acc[u][r];  // the mirrored tile
              }
            }
          }
        }
        rsum = block_sum(rsum, wred);
        if (tid == 0) out[rec_r] = rsum;
      }
      if (!ps_grid_sync(g.bar, nblk, epoch, g.spin_limit, g.status, &s_fail)) return;
      // ---- B: fixed-order sum of the records, element slices over the work-groups ------
      {
        const int nv = rec_r + 1;
        const int per = (nv + G - 1) / G;
        const int e0 = (int)blockIdx.x * per;
        const int e1 = min(nv, e0 + per);
        double* cb = U + g.ubuf;  // kPsThreads doubles
        for (int base = e0; base < e1; base += kPsThreads) {
          const int cnt = min(e1 - base, kPsThreads);
          const int ngrp = kPsThreads / cnt;
          const int le = tid % cnt, grp = tid / cnt;
          double acc = 0.0;
          if (grp < ngrp)
            for (int r = grp; r < nrec; r += ngrp) acc += g.part[(int64_t)r * g.rec + base + le];
          cb[tid] = acc;
          __syncthreads();
          if (tid < cnt) {
            double t = 0.0;
            for (int qq = 0; qq < ngrp; ++qq) t += cb[qq * cnt + tid];
            g.red[base + tid] = t;
          }
          __syncthreads();
        }
      }
      if (!ps_grid_sync(g.bar, nblk, epoch, g.spin_limit, g.status, &s_fail)) return;
      // ---- C: the error of the sweep before, the stopping test, the solve ---------------
      if (report) {
        const double e = sqrt(g.red[rec_r] / pn2);
        if (blockIdx.x == 0 && tid == 0) {
          g.trace[s - 1] = e;
          *g.sweeps_run = s;
        }
        if (g.tol > 0.0 && s >= 2 && fabs(e - eprev) < g.tol) stop = true;
        eprev = e;
        if (stop || last) break;
      }
      {
        // the next update's first P tile, in flight during the solve
        const int nn = n + 1 < N ? n + 1 : 0;
        const PsGeom qn = ps_geom(g, nn, TJ);
        double* rowbuf = U + g.ubuf;
        double* colbuf = rowbuf + 2 * 4 * kPsSolveW;
        auto prefetch = [&]() { ps_load_p<TJ, KPER>(g, qn, blockIdx.x, pv); };
        if (!ps_solve<8, TPW, kPsSolveW>(g.red, g.red + rec_g, RR, Kn, 0, Kn, Rb, Zs + q.zoffN,
                                          rowbuf, colbuf, prefetch) &&
            blockIdx.x == 0 && tid == 0)
          atomicOr(g.status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
        __syncthreads();
      }
    }
  }
  if (blockIdx.x == 0)
    for (int x = tid; x < (int)g.ztotal; x += kPsThreads) g.Z[x] = Zs[x];
}

__global__ void als_persist_begin_kernel(unsigned* bar, int* sweeps_run) {
  *bar = 0u;
  *sweeps_run = 0;
}

namespace {
// Tile buffers (B, the P tile, core n reshaped) and, past them, the buffers of the record sum
// and the solve.
int64_t ps_ubuf(int TJ, int maxK, int maxRR) {
  const int ldB = pad16(maxRR) + 1;
  return (int64_t)TJ * ldB + (int64_t)pad16(maxK) * (TJ + 1) + (int64_t)pad16(maxK) * ldB;
}

int64_t ps_words(int TJ, int maxK, int maxRR, int64_t ztotal) {
  const int64_t c = std::max<int64_t>(2 * 4 * kPsSolveW + 2 * kPsSolveW * 4, kPsThreads);
  return zwords(ztotal) + ps_ubuf(TJ, maxK, maxRR) + c;
}

template <int RM, int TPW, int KT>
const void* ps_fn3(int TJ) {
  return TJ == 128 ? (const void*)als_persist_kernel<RM, TPW, 128, KT>
                   : (const void*)als_persist_kernel<RM, TPW, 64, KT>;
}

template <int RM, int TPW>
const void* ps_fn2(int TJ, int maxK) {
  return maxK <= 32 ? ps_fn3<RM, TPW, 32>(TJ) : ps_fn3<RM, TPW, 64>(TJ);
}

template <int RM>
const void* ps_fn(int TJ, int tpw, int maxK) {
  return tpw == 1 ? ps_fn2<RM, 1>(TJ, maxK) : tpw == 2 ? ps_fn2<RM, 2>(TJ, maxK)
                                                       : ps_fn2<RM, 4>(TJ, maxK);
}
}  // namespace

// Plans the single launch; false if the shape is outside what it takes (the caller then runs
// the two-kernel updates).  Fills TJ, G, rec, maxNe, rmax and the LDS bytes.
bool als_persist_plan(AlsPersistArgs* g, size_t* lds) {
  int maxK = 0, rmax = 0, maxRR = 0, maxNe = 0;
  int64_t rec = 1;
  for (int n = 0; n < g->N; ++n) {
    const int Kn = g->K[n], RR = g->R[n] * g->R[(n + 1) % g->N];
    maxK = std::max(maxK, Kn);
    rmax = std::max(rmax, g->R[n]);
    maxRR = std::max(maxRR, RR);
    if (RR > 64 || !ps_tpw(RR, Kn)) return false;
    maxNe = std::max(maxNe, ps_tpw(RR, Kn));
    rec = std::max(rec, (int64_t)Kn * RR + (int64_t)RR * RR + 1);
  }
  if (rmax > 8 || maxK > 64 || g->ztotal > kZldsMax || g->total >= (1LL << 31)) return false;
  {  // output tiles of M and the Gram per wavefront
    const int NT = pad16(maxRR) / 16, MT = pad16(maxK) / 16;
    if (MT * NT + NT * (NT + 1) / 2 > 8 * kPsTiles) return false;
  }
  int tj = 0;
  for (int t = 128; t >= 64; t /= 2)
    if (ps_words(t, maxK, maxRR, g->ztotal) * 8 <= 150 * 1024) {
      tj = t;
      break;
    }
  if (!tj) return false;
  g->TJ = tj;
  int64_t maxTiles = 1;
  for (int n = 0; n < g->N; ++n) {
    const int64_t J = g->total / g->K[n];
    maxTiles = std::max(maxTiles, (J + tj - 1) / tj);
  }
  g->G = (int)std::min<int64_t>(maxTiles, 128);
  g->rec = rec;
  g->maxNe = maxNe;
  g->rmax = rmax;
  g->maxK = maxK;
  g->ubuf = ps_ubuf(tj, maxK, maxRR);
  *lds = (size_t)ps_words(tj, maxK, maxRR, g->ztotal) * 8;
  return true;
}

hipError_t launch_als_persist(const AlsPersistArgs& ga, size_t lds, hipStream_t s) {
  AlsPersistArgs g = ga;
  // maxNe holds the largest tiles-per-wavefront tier of the solve over the updates
  const void* fn = g.rmax <= 4 ? ps_fn<4>(g.TJ, g.maxNe, g.maxK)
                 : g.rmax <= 6 ? ps_fn<6>(g.TJ, g.maxNe, g.maxK)
                               : ps_fn<8>(g.TJ, g.maxNe, g.maxK);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPsThreads, lds)) != hipSuccess)
    return e;
  if ((int64_t)per_cu * cus < g.G) return hipErrorCooperativeLaunchTooLarge;
  hipLaunchKernelGGL(als_persist_begin_kernel, dim3(1), dim3(1), 0, s, g.bar, g.sweeps_run);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin("als_persist", s);
  void* args[] = {&g};
  e = hipLaunchCooperativeKernel(fn, dim3((unsigned)g.G), dim3(kPsThreads), args, (unsigned)lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
