// TR-ALS (Alg. 1 step 9) with two kernels per core update.
//
// als_accum   columns j of P_<n> in tiles of 32: each tile's subchain rows
//             B[j, a*R_{n+1} + b] = S_j[b, a] are formed in LDS from the current cores
//             (one row b of S_j per thread, a vector-matrix product per core), then
//             M += P_<n>[:, tile] B_tile and Gram += B_tile^T B_tile accumulate in
//             registers.  Optionally the same tile also gives ||P - Psi(Z)||^2 with the
//             current core n (Psi_<n> = Z_{n,(2)} B^T): the first update of a sweep reports
//             the error of the sweep before it at no extra pass.
// als_solve   one work-group: fixed-order sum of the partials into LDS, FP64 Cholesky of
//             the Gram matrix (one wavefront when R_n R_{n+1} <= 64), forward and back
//             substitution for every row of M (16 lanes per right-hand side), new core.
//             It also closes the previous sweep: error = sqrt(residual / ||P||^2), the
//             stopping test, and the device flag that turns every later kernel into a no-op.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kA2TJ = 32;

// Orders the LDS accesses of one wavefront (the lanes of a wave run in lockstep).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int kA2Threads = 1024;

// Outputs of the per-column accumulation: [M (Kn x RR); Gram (RR x RR) if direct], as the
// product L B_tile with L = [P_<n>[:, tile]; B_tile^T].  Thread t owns outputs t + 1024 q.
// TJ columns per tile: 128 when the Gram comes from transfer matrices (every thread then
// forms a subchain row), 32 when the Gram is accumulated here.
template <int RM, int NQ, int TJ>
__global__ __launch_bounds__(kA2Threads) void als_accum_kernel(AlsArgs2 g) {
  extern __shared__ __align__(16) double sm[];
  const int RR = g.RR, Kn = g.Kn, Ra = g.Ra, Rb = g.Rb;
  double* Zs = sm;                                          // packed cores (zlds)
  double* Bs = sm + (g.zlds ? (g.ztotal + 1) / 2 * 2 : 0);  // [TJ][RR]
  double* Ls = Bs + TJ * RR;                                // [Kn + RR?][TJ]
  const double* Zsrc = g.zlds ? Zs : g.Z;
  __shared__ double red[32];
  const int nM = Kn * RR;
  const int nout = nM + (g.gram_direct ? RR * RR : 0);
  const bool accum = g.mode & 1, resid = g.mode & 2;
  const int tid = threadIdx.x;
  if (g.zlds) {  // cores: all loads issued before any store (at most 6 per thread)
    double zt[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int64_t x = tid + (int64_t)e * kA2Threads;
      zt[e] = x < g.ztotal ? g.Z[x] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int64_t x = tid + (int64_t)e * kA2Threads;
      if (x < g.ztotal) Zs[x] = zt[e];
    }
  }
  if (*g.done) return;
  double acc[NQ];
  int rowoff[NQ], colidx[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = 0.0;
    const int o = tid + q * kA2Threads;
    rowoff[q] = (o < nout) ? (o / RR) * TJ : -1;
    colidx[q] = o % RR;
  }
  double rsum = 0.0;
  const int64_t ntiles = (g.J + TJ - 1) / TJ;
  const int64_t t0 = (int64_t)blockIdx.x * g.tiles_per_wg;
  const int64_t t1 = min(ntiles, t0 + g.tiles_per_wg);
  __syncthreads();
  for (int64_t t = t0; t < t1; ++t) {
    const int j0 = (int)(t * TJ);
    const int jn = (int)min((int64_t)TJ, g.J - j0);
    // P_<n>[:, tile] (column bases in int32: P has < 2^31 entries); all loads issued first
    {
      constexpr int kPer = (64 * TJ + kA2Threads - 1) / kA2Threads;
      double pv[kPer];
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int x = tid + e * kA2Threads;
        const int i = x / TJ, jj = x % TJ;
        pv[e] = 0.0;
        if (x < Kn * TJ && jj < jn) {
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
        const int x = tid + e * kA2Threads;
        if (x < Kn * TJ) Ls[x] = pv[e];
      }
    }
    // subchain rows: thread (jl, b) forms row b of S_j
    for (int x = tid; x < TJ * Rb; x += kA2Threads) {
      const int jl = x / Rb, b = x % Rb;
      double v[RM], w[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = (jl < jn && a == b) ? 1.0 : 0.0;
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
        int cur = Rb;
#pragma unroll
        for (int u = 0; u < 7; ++u) {
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
      for (int a = 0; a < RM; ++a) {
        if (a < Ra) {
          const int r = a * Rb + b;
          Bs[jl * RR + r] = v[a];
          if (g.gram_direct) Ls[(Kn + r) * TJ + jl] = v[a];
        }
      }
    }
    __syncthreads();
    if (accum) {
#pragma unroll 8
      for (int jj = 0; jj < TJ; ++jj) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (rowoff[q] >= 0) acc[q] += Ls[rowoff[q] + jj] * Bs[jj * RR + colidx[q]];
      }
    }
    if (resid) {
      const double* Zn = Zsrc + g.zoffN;
      for (int x = tid; x < Kn * TJ; x += kA2Threads) {
        const int i = x / TJ, jj = x % TJ;
        if (jj < jn) {
          double psi = 0.0;
          for (int a = 0; a < Ra; ++a) {
            const double* zr = Zn + (a * Kn + i) * Rb;
            const double* br = Bs + jj * RR + a * Rb;
#pragma unroll 8
            for (int b = 0; b < Rb; ++b) psi += zr[b] * br[b];
          }
          const double d = Ls[x] - psi;
          rsum += d * d;
        }
      }
    }
    __syncthreads();
  }
  double* out = g.part + (int64_t)blockIdx.x * (nout + 1);
  if (accum) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (rowoff[q] >= 0) out[tid + q * kA2Threads] = acc[q];
  }
  rsum = block_sum(rsum, red);
  if (tid == 0) out[nout] = rsum;
}


// Cholesky of the RR x RR matrix G (LDS, row-major) by one wavefront, RR <= RMAX <= 64:
// lane i keeps row i in registers (loops unrolled to RMAX so every index is static); at
// step j the pivot and column j are read from the owning lanes with readlane.  The lower
// factor is written back to G.  Sets *failed when a pivot is not positive.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int2 p = __builtin_bit_cast(int2, v);
  int2 q;
  q.x = __builtin_amdgcn_readlane(p.x, lane);
  q.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, q);
}

template <int RMAX>
__device__ void chol_wave(double* G, int RR, int* failed) {
  const int i = threadIdx.x & 63;
  double row[RMAX];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) row[c] = (i < RR && c < RR) ? G[i * RR + c] : 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    if (j < RR && ok) {
      const double d = readlane_f64(row[j], j);
      if (!(d > 0.0)) {
        ok = false;
      } else {
        const double ljj = sqrt(d);
        const double inv = 1.0 / ljj;
        if (i == j) row[j] = ljj;
        if (i > j) row[j] *= inv;
#pragma unroll
        for (int k = j + 1; k < RMAX; ++k) {
          if (k < RR) {
            const double lkj = readlane_f64(row[j], k);
            if (i >= k) row[k] -= row[j] * lkj;
          }
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // keep each step's loads and readlanes local
  }
  if (!ok) {
    if (i == 0) *failed = 1;
    return;
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c)
    if (i < RR && c <= i && c < RR) G[i * RR + c] = row[c];
}

// Forward and back substitution with the factor L (lower part of G) for every row of M
// (Kn x RR, LDS): lane/thread r owns row r in registers; L is read with uniform addresses.
template <int RMAX>
__device__ void subst_rows(double* M, const double* G, int RR, int Kn) {
  for (int row = threadIdx.x; row < Kn; row += blockDim.x) {
    double m[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) m[c] = c < RR ? M[row * RR + c] : 0.0;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < RR) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < r; ++k) {
          if (k & 1)
            s1 += G[r * RR + k] * m[k];
          else
            s0 += G[r * RR + k] * m[k];
        }
        m[r] = (m[r] - (s0 + s1)) / G[r * RR + r];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = RMAX - 1; r >= 0; --r) {
      if (r < RR) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = r + 1; k < RMAX; ++k) {
          if (k < RR) {
            if (k & 1)
              s1 += G[k * RR + r] * m[k];
            else
              s0 += G[k * RR + r] * m[k];
          }
        }
        m[r] = (m[r] - (s0 + s1)) / G[r * RR + r];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
      if (c < RR) M[row * RR + c] = m[c];
  }
}

// ---------------------------------------------------------------------------------------
// RMAX: register bound of the Cholesky and substitutions (16, 36, 64); 0 = LDS fallback.
template <int RMAX>
__global__ __launch_bounds__(512) void als_solve2_kernel(AlsSolveArgs g) {
  if (*g.done) return;
  extern __shared__ __align__(16) double sm[];
  const int RR = g.RR, Kn = g.Kn, nM = Kn * RR, nout = nM + RR * RR;
  double* M = sm;        // Kn x RR, overwritten by the solution rows
  double* G = sm + nM;   // RR x RR, lower Cholesky factor in place
  __shared__ double red[16];
  __shared__ int failed;
  const int tid = threadIdx.x, nth = blockDim.x;
  // close the previous sweep: its error was accumulated by the partials of this update
  const int nstore = g.gram_direct ? nout : nM;  // partial record length (+1 residual)
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
  const int nred = g.gram_direct ? nout : nM;  // outputs summed from the partials
  for (int o = tid; o < nred; o += nth) {
    const double* src = g.part + o;
    const int64_t st = nred + 1;
    double s = 0.0;
    int c = 0;
    for (; c + 16 <= g.nparts; c += 16) {  // sixteen loads in flight, summed in order
      double v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = src[(c + e) * st];
#pragma unroll
      for (int e = 0; e < 16; ++e) s += v[e];
    }
    for (; c < g.nparts; ++c) s += src[c * st];
    sm[o] = s;
  }
  if (tid == 0) failed = 0;
  if (!g.gram_direct) {
    // Gram from transfer matrices: sum_j S_j (x) S_j = E_{n+1} E_{n+2} ... E_{n-1},
    // E_m[(p,p'),(q,q')] = sum_i Z_m[p,i,q] Z_m[p',i,q']; then Gram[(a,b),(a',b')] is the
    // entry [(b,b'),(a,a')] of that product.
    double* Tm = sm + nout;            // running product, R_{n+1}^2 x R_cur^2
    double* Em = Tm + g.tsz;           // next transfer matrix
    double* Tn = Em + g.tsz;           // product buffer
    double* Zs = Tn + g.tsz;           // cores (one batch of loads)
    {
      double zt[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) {
        const int64_t x = tid + (int64_t)e * nth;
        zt[e] = x < g.ztotal ? g.Z[x] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 12; ++e) {
        const int64_t x = tid + (int64_t)e * nth;
        if (x < g.ztotal) Zs[x] = zt[e];
      }
    }
    __syncthreads();
    const int Rn1 = g.Rc[(g.n + 1) % g.N];
    int rcur = Rn1;
    for (int t = 1; t < g.N; ++t) {
      const int m = (g.n + t) % g.N;
      const int Rp = g.Rc[m], Rq = g.Rc[(m + 1) % g.N], Km = g.Kc[m];
      const double* Zm = Zs + g.zoff[m];
      double* dst = (t == 1) ? Tm : Em;
      const int ne = Rp * Rp * Rq * Rq;
      for (int x = tid; x < ne; x += nth) {
        const int col = x % (Rq * Rq), row = x / (Rq * Rq);
        const int p = row / Rp, pp = row % Rp, q = col / Rq, qq = col % Rq;
        const double* za = Zm + p * Km * Rq + q;
        const double* zb = Zm + pp * Km * Rq + qq;
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < Km; ++i) s += za[i * Rq] * zb[i * Rq];
        dst[x] = s;
      }
      __syncthreads();
      if (t > 1) {
        const int nr = Rn1 * Rn1, nk = Rp * Rp, nc = Rq * Rq;
        for (int x = tid; x < nr * nc; x += nth) {
          const int r = x / nc, c = x % nc;
          double s = 0.0;
#pragma unroll 8
          for (int k = 0; k < nk; ++k) s += Tm[r * nk + k] * Em[k * nc + c];
          Tn[x] = s;
        }
        __syncthreads();
        for (int x = tid; x < nr * nc; x += nth) Tm[x] = Tn[x];
        __syncthreads();
      }
      rcur = Rq;
    }
    (void)rcur;
    // here rcur == R_n: Tm is R_{n+1}^2 x R_n^2
    const int Rb2 = g.Rb, Ra2 = g.Ra;
    for (int x = tid; x < RR * RR; x += nth) {
      const int r1 = x / RR, r2 = x % RR;           // (a,b), (a',b')
      const int a = r1 / Rb2, b = r1 % Rb2, a2 = r2 / Rb2, b2 = r2 % Rb2;
      sm[nM + x] = Tm[(b * Rb2 + b2) * (Ra2 * Ra2) + (a * Ra2 + a2)];
    }
  }
  __syncthreads();
  if constexpr (RMAX > 0) {
    if (tid < 64) chol_wave<RMAX>(G, RR, &failed);
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
  }
  __syncthreads();
  if (failed) {
    if (tid == 0) atomicOr(g.status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
    return;
  }
  // one lane per right-hand side (a row m of M): L y = m, then L^T w = y
  if constexpr (RMAX > 0) {
    subst_rows<RMAX>(M, G, RR, Kn);
  } else {
    for (int row = tid; row < Kn; row += nth) {
      double* m = M + (int64_t)row * RR;
      for (int r = 0; r < RR; ++r) {
        double sacc = 0.0;
        for (int k = 0; k < r; ++k) sacc += G[r * RR + k] * m[k];
        m[r] = (m[r] - sacc) / G[r * RR + r];
      }
      for (int r = RR - 1; r >= 0; --r) {
        double sacc = 0.0;
        for (int k = r + 1; k < RR; ++k) sacc += G[k * RR + r] * m[k];
        m[r] = (m[r] - sacc) / G[r * RR + r];
      }
    }
  }
  __syncthreads();
  for (int x = tid; x < nM; x += nth) {
    const int i = x / RR, r = x % RR;
    const int a = r / g.Rb, b = r % g.Rb;
    g.Zn[((int64_t)a * Kn + i) * g.Rb + b] = M[x];
  }
}

// ---------------------------------------------------------------------------------------
static int64_t zlds_words(int64_t ztotal) { return (ztotal + 1) / 2 * 2; }
constexpr int64_t kZldsMax = 6144;  // cores staged in LDS up to 48 KB (6 loads per thread)

static int accum_tj(int gram_direct) { return gram_direct ? 32 : 128; }

size_t als2_accum_lds(int Kn, int RR, int64_t ztotal, int gram_direct) {
  const int TJ = accum_tj(gram_direct);
  const int64_t z = ztotal <= kZldsMax ? zlds_words(ztotal) : 0;
  return (size_t)(z + TJ * RR + (Kn + (gram_direct ? RR : 0)) * TJ) * sizeof(double);
}
size_t als2_solve_lds(int Kn, int RR, int tsz, int gram_direct, int64_t ztotal) {
  return (size_t)(Kn * RR + RR * RR + (gram_direct ? 0 : 3 * tsz + ztotal)) * sizeof(double);
}

bool als2_supported(int Kn, int RR, int Rb, int64_t J, int64_t ztotal, int gram_direct, int tsz) {
  const int64_t nout = (int64_t)Kn * RR + (gram_direct ? (int64_t)RR * RR : 0);
  return Kn <= 64 && J < (1LL << 31) &&
         nout <= 16LL * kA2Threads &&
         als2_accum_lds(Kn, RR, ztotal, gram_direct) <= 150 * 1024 &&
         als2_solve_lds(Kn, RR, tsz, gram_direct, ztotal) <= 150 * 1024;
}

int64_t als2_grid(int64_t J, int gram_direct) {
  const int TJ = accum_tj(gram_direct);
  const int64_t ntiles = (J + TJ - 1) / TJ;
  int64_t g = gram_direct ? ntiles / 4 : ntiles;
  if (g < 1) g = 1;
  if (g > 32) g = 32;
  const int64_t per = (ntiles + g - 1) / g;
  return (ntiles + per - 1) / per;
}

template <int RM, int TJ>
static const void* accum_fn(int nq) {
  if (nq <= 1) return (const void*)als_accum_kernel<RM, 1, TJ>;
  if (nq <= 2) return (const void*)als_accum_kernel<RM, 2, TJ>;
  if (nq <= 4) return (const void*)als_accum_kernel<RM, 4, TJ>;
  if (nq <= 8) return (const void*)als_accum_kernel<RM, 8, TJ>;
  return (const void*)als_accum_kernel<RM, 16, TJ>;
}

template <int TJ>
static const void* accum_pick(int rmax, int nq) {
  return rmax <= 8 ? accum_fn<8, TJ>(nq) : rmax <= 16 ? accum_fn<16, TJ>(nq)
                                                      : accum_fn<RTR_MAX_RANK, TJ>(nq);
}

hipError_t launch_als_accum(AlsArgs2 g, int64_t grid, int rmax, hipStream_t s) {
  const int TJ = accum_tj(g.gram_direct);
  const int64_t ntiles = (g.J + TJ - 1) / TJ;
  g.tiles_per_wg = (ntiles + grid - 1) / grid;
  g.zlds = g.ztotal <= kZldsMax;
  const size_t lds = als2_accum_lds(g.Kn, g.RR, g.ztotal, g.gram_direct);
  const int nout = g.Kn * g.RR + (g.gram_direct ? g.RR * g.RR : 0);
  const int nq = (nout + kA2Threads - 1) / kA2Threads;
  const void* fn = g.gram_direct ? accum_pick<32>(rmax, nq) : accum_pick<128>(rmax, nq);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("als_accum", s);
  void* args[] = {&g};
  e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kA2Threads), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_als_solve2(AlsSolveArgs g, hipStream_t s) {
  const size_t lds = als2_solve_lds(g.Kn, g.RR, g.tsz, g.gram_direct, g.ztotal);
  const void* fn = g.RR <= 16 ? (const void*)als_solve2_kernel<16>
                 : g.RR <= 36 ? (const void*)als_solve2_kernel<36>
                 : g.RR <= 64 ? (const void*)als_solve2_kernel<64>
                              : (const void*)als_solve2_kernel<0>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("als_solve", s);
  void* args[] = {&g};
  e = hipLaunchKernel(fn, dim3(1), dim3(512), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
