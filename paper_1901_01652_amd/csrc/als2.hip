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
constexpr int kA2Acc = 64;
constexpr int kA2Threads = 256;

// Left operand L = [P_<n>[:, tile] (Kn rows); B_tile^T (RR rows)] and right operand B_tile:
// [M; Gram] += L B_tile, output (Kn + RR) x RR.  Thread t owns outputs t + 256 q, q < NQ.
template <int RM, int NQ>
__global__ __launch_bounds__(kA2Threads) void als_accum_kernel(AlsArgs2 g) {
  if (*g.done) return;
  extern __shared__ __align__(16) double sm[];
  const int RR = g.RR, Kn = g.Kn, Ra = g.Ra, Rb = g.Rb;
  double* Bs = sm;                         // [32][RR]
  double* Ls = sm + kA2TJ * RR;            // [Kn + RR][32]
  __shared__ int64_t pbase[kA2TJ];
  __shared__ double red[16];
  const int nM = Kn * RR, nout = nM + RR * RR;
  const bool accum = g.mode & 1, resid = g.mode & 2;
  const double* Zn = g.Z + g.zoffN;
  const int tid = threadIdx.x;
  double acc[NQ];
  int rowoff[NQ], colidx[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = 0.0;
    const int o = tid + q * kA2Threads;
    rowoff[q] = (o < nout) ? (o / RR) * kA2TJ : -1;
    colidx[q] = o % RR;
  }
  double rsum = 0.0;
  const int64_t ntiles = (g.J + kA2TJ - 1) / kA2TJ;
  const int64_t t0 = (int64_t)blockIdx.x * g.tiles_per_wg;
  const int64_t t1 = min(ntiles, t0 + g.tiles_per_wg);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t j0 = t * kA2TJ;
    const int jn = (int)min((int64_t)kA2TJ, g.J - j0);
    // subchain rows: thread (jl, b) forms row b of S_j
    for (int x = tid; x < kA2TJ * Rb; x += kA2Threads) {
      const int jl = x / Rb, b = x % Rb;
      double v[RM], w[RM];
#pragma unroll
      for (int a = 0; a < RM; ++a) v[a] = (jl < jn && a == b) ? 1.0 : 0.0;
      if (jl < jn) {
        int64_t rem = j0 + jl;
        int cur = Rb;
        int idx0 = 0, idx1 = 0, idx2 = 0, idx3 = 0, idx4 = 0, idx5 = 0, idx6 = 0;
        {
          int tmp[7];
          for (int u = g.N - 2; u >= 0; --u) {
            tmp[u] = (int)(rem % g.chI[u]);
            rem /= g.chI[u];
          }
          idx0 = tmp[0];
          if (g.N > 2) idx1 = tmp[1];
          if (g.N > 3) idx2 = tmp[2];
          if (g.N > 4) idx3 = tmp[3];
          if (g.N > 5) idx4 = tmp[4];
          if (g.N > 6) idx5 = tmp[5];
          if (g.N > 7) idx6 = tmp[6];
        }
        for (int u = 0; u < g.N - 1; ++u) {
          const int iu = u == 0 ? idx0 : u == 1 ? idx1 : u == 2 ? idx2 : u == 3 ? idx3
                       : u == 4 ? idx4 : u == 5 ? idx5 : idx6;
          const int cRb = g.chRb[u];
          const double* G = g.Z + g.chOff[u] + (int64_t)iu * cRb;
          const int64_t rs = (int64_t)g.chI[u] * cRb;
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
#pragma unroll
      for (int a = 0; a < RM; ++a) {
        if (a < Ra) {
          const int r = a * Rb + b;
          Bs[jl * RR + r] = v[a];
          Ls[(Kn + r) * kA2TJ + jl] = v[a];
        }
      }
    }
    if (tid < kA2TJ) pbase[tid] = (tid < jn) ? cyc_base_of(g.N, g.cycK, g.cycStride, j0 + tid) : (int64_t)-1;
    __syncthreads();
    for (int x = tid; x < Kn * kA2TJ; x += kA2Threads) {
      const int i = x / kA2TJ, jj = x % kA2TJ;
      const int64_t pb = pbase[jj];
      Ls[x] = (pb >= 0) ? g.P[pb + (int64_t)i * g.strideN] : 0.0;
    }
    __syncthreads();
    if (accum) {
      for (int jj = 0; jj < kA2TJ; ++jj) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (rowoff[q] >= 0) acc[q] += Ls[rowoff[q] + jj] * Bs[jj * RR + colidx[q]];
      }
    }
    if (resid) {
      for (int x = tid; x < Kn * kA2TJ; x += kA2Threads) {
        const int i = x / kA2TJ, jj = x % kA2TJ;
        if (jj < jn) {
          double psi = 0.0;
          for (int a = 0; a < Ra; ++a)
            for (int b = 0; b < Rb; ++b)
              psi += Zn[((int64_t)a * Kn + i) * Rb + b] * Bs[jj * RR + a * Rb + b];
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

// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void als_solve2_kernel(AlsSolveArgs g) {
  if (*g.done) return;
  extern __shared__ __align__(16) double sm[];
  const int RR = g.RR, Kn = g.Kn, nM = Kn * RR, nout = nM + RR * RR;
  double* M = sm;        // Kn x RR, overwritten by the solution rows
  double* G = sm + nM;   // RR x RR, lower Cholesky factor in place
  __shared__ double red[16];
  __shared__ int failed;
  const int tid = threadIdx.x, nth = blockDim.x;
  // close the previous sweep: its error was accumulated by the partials of this update
  if (g.report_sweep >= 0) {
    double s = 0.0;
    for (int c = tid; c < g.nparts; c += nth) s += g.part[(int64_t)c * (nout + 1) + nout];
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
  for (int o = tid; o < nout; o += nth) {
    double s = 0.0;
    for (int c = 0; c < g.nparts; ++c) s += g.part[(int64_t)c * (nout + 1) + o];
    sm[o] = s;
  }
  if (tid == 0) failed = 0;
  __syncthreads();
  if (RR <= 64) {
    // one wavefront: lane i owns row i of the factor
    if (tid < 64) {
      const int i = tid;
      for (int j = 0; j < RR; ++j) {
        double d = 0.0;
        if (i == j) {
          d = G[j * RR + j];
          for (int k = 0; k < j; ++k) d -= G[j * RR + k] * G[j * RR + k];
          G[j * RR + j] = (d > 0.0) ? sqrt(d) : 0.0;
        }
        const double djj = __shfl(d, j, 64);
        if (!(djj > 0.0)) {
          if (i == 0) failed = 1;
          break;
        }
        wave_sync();
        if (i > j && i < RR) {
          double s = G[i * RR + j];
          for (int k = 0; k < j; ++k) s -= G[i * RR + k] * G[j * RR + k];
          G[i * RR + j] = s / G[j * RR + j];
        }
        wave_sync();
      }
    }
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
  // 16 lanes per right-hand side: L y = m, then L^T w = y
  const int grp = tid >> 4, l16 = tid & 15, ngrp = nth >> 4;
  for (int row = grp; row < Kn; row += ngrp) {
    double* m = M + (int64_t)row * RR;
    for (int r = 0; r < RR; ++r) {
      double s = 0.0;
      for (int k = l16; k < r; k += 16) s -= G[r * RR + k] * m[k];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      if (l16 == 0) m[r] = (m[r] + s) / G[r * RR + r];
      wave_sync();
    }
    for (int r = RR - 1; r >= 0; --r) {
      double s = 0.0;
      for (int k = r + 1 + l16; k < RR; k += 16) s -= G[k * RR + r] * m[k];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      if (l16 == 0) m[r] = (m[r] + s) / G[r * RR + r];
      wave_sync();
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
size_t als2_accum_lds(int Kn, int RR) { return (size_t)(kA2TJ * RR + (Kn + RR) * kA2TJ) * sizeof(double); }
size_t als2_solve_lds(int Kn, int RR) { return (size_t)(Kn * RR + RR * RR) * sizeof(double); }

bool als2_supported(int Kn, int RR) {
  return Kn <= 64 && (int64_t)Kn * RR + (int64_t)RR * RR <= (int64_t)kA2Threads * kA2Acc &&
         als2_accum_lds(Kn, RR) <= 150 * 1024 && als2_solve_lds(Kn, RR) <= 150 * 1024;
}

int64_t als2_grid(int64_t J) {
  const int64_t ntiles = (J + kA2TJ - 1) / kA2TJ;
  int64_t g = ntiles / 4;
  if (g < 1) g = 1;
  if (g > 64) g = 64;
  const int64_t per = (ntiles + g - 1) / g;
  return (ntiles + per - 1) / per;
}

template <int RM>
static const void* accum_fn(int nq) {
  if (nq <= 8) return (const void*)als_accum_kernel<RM, 8>;
  if (nq <= 16) return (const void*)als_accum_kernel<RM, 16>;
  if (nq <= 32) return (const void*)als_accum_kernel<RM, 32>;
  return (const void*)als_accum_kernel<RM, 64>;
}

hipError_t launch_als_accum(AlsArgs2 g, int64_t grid, int rmax, hipStream_t s) {
  const int64_t ntiles = (g.J + kA2TJ - 1) / kA2TJ;
  g.tiles_per_wg = (ntiles + grid - 1) / grid;
  const size_t lds = als2_accum_lds(g.Kn, g.RR);
  const int nout = g.Kn * g.RR + g.RR * g.RR;
  const int nq = (nout + kA2Threads - 1) / kA2Threads;
  const void* fn = rmax <= 8 ? accum_fn<8>(nq) : rmax <= 16 ? accum_fn<16>(nq) : accum_fn<RTR_MAX_RANK>(nq);
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
  const size_t lds = als2_solve_lds(g.Kn, g.RR);
  hipError_t e = hipFuncSetAttribute((const void*)als_solve2_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  prof_begin("als_solve", s);
  void* args[] = {&g};
  e = hipLaunchKernel((const void*)als_solve2_kernel, dim3(1), dim3(1024), args, lds, s);
  prof_end(s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace rtr
