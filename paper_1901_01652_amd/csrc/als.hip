// Alg. 1 step 9 with TR-ALS on the projected tensor P (FP64).
//
// Core n is the least-squares solution of Eq. (2) on P:
//   P_<n> ~ Z_{n,(2)} B^T,  B[j, a*R_{n+1} + b] = S_j[b, a],
//   S_j = Z_{n+1}(i_{n+1}) ... Z_N(i_N) Z_1(i_1) ... Z_{n-1}(i_{n-1})   (subchain, Sec. 2.2)
// solved through the normal equations (B^T B) Z_{n,(2)}^T = B^T P_<n>^T:
//   chain_kernel      B (one row of S_j per thread)
//   als_partial       per chunk of columns j: M = P_<n> B and Gram = B^T B
//   als_reduce        fixed-order sum of the chunk partials
//   als_solve         FP64 Cholesky of the Gram matrix, triangular solves, new core
//   als_resid/err     after each sweep ||P - Psi(Z)||^2 from the last update's B, the
//                     relative error, and the stopping test (a device flag that turns
//                     every later kernel of the decomposition into a no-op)
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kRMax = RTR_MAX_RANK;

// ---------------------------------------------------------------------------------------
template <int RM>
__global__ __launch_bounds__(256) void chain_kernel(Chain ch, int64_t count, int transpose,
                                                    double* __restrict__ out,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  const int R0 = ch.Ra[0];
  const int RL = ch.Rb[ch.L - 1];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count * R0) return;
  int64_t l = p / R0;
  const int r0 = (int)(p % R0);
  const int64_t lrow = l;
  int idx[8];
  for (int t = ch.L - 1; t >= 0; --t) {
    idx[t] = (int)(l % ch.I[t]);
    l /= ch.I[t];
  }
  double v[RM], w[RM];
#pragma unroll
  for (int a = 0; a < RM; ++a) v[a] = (a == r0) ? 1.0 : 0.0;
  int cur = R0;
  for (int t = 0; t < ch.L; ++t) {
    const int Ra = ch.Ra[t], Rb = ch.Rb[t];
    const double* G = ch.core[t] + (int64_t)idx[t] * Rb;
    const int64_t rowstride = (int64_t)ch.I[t] * Rb;
#pragma unroll
    for (int b = 0; b < RM; ++b) w[b] = 0.0;
#pragma unroll
    for (int a = 0; a < RM; ++a) {
      if (a < cur) {
        const double va = v[a];
        const double* g = G + a * rowstride;
#pragma unroll
        for (int b = 0; b < RM; ++b)
          if (b < Rb) w[b] += va * g[b];
      }
    }
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = w[b];
    cur = Rb;
    (void)Ra;
  }
  double* o = out + lrow * (int64_t)(R0 * RL);
#pragma unroll
  for (int c = 0; c < RM; ++c) {
    if (c < RL) {
      if (transpose)
        o[c * R0 + r0] = v[c];
      else
        o[r0 * RL + c] = v[c];
    }
  }
}

hipError_t launch_chain(const Chain& ch, int64_t count, int transpose, double* out,
                        const int* done, hipStream_t s) {
  int rmax = 0;
  for (int t = 0; t < ch.L; ++t) rmax = max(rmax, max(ch.Ra[t], ch.Rb[t]));
  const int64_t n = count * ch.Ra[0];
  const unsigned blocks = (unsigned)((n + 255) / 256);
  prof_begin("chain", s);
  if (rmax <= 8)
    hipLaunchKernelGGL(chain_kernel<8>, dim3(blocks), dim3(256), 0, s, ch, count, transpose,
                       out, done);
  else if (rmax <= 16)
    hipLaunchKernelGGL(chain_kernel<16>, dim3(blocks), dim3(256), 0, s, ch, count, transpose,
                       out, done);
  else
    hipLaunchKernelGGL(chain_kernel<kRMax>, dim3(blocks), dim3(256), 0, s, ch, count,
                       transpose, out, done);
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
constexpr int kAlsTJ = 16;
constexpr int kAlsAcc = 64;  // outputs per thread
constexpr int kAlsThreads = 256;
// outputs per work-group: the Kn*RR + RR*RR outputs are split into blocks of this many along
// the grid's second dimension
constexpr int kAlsOutBlk = kAlsThreads * kAlsAcc;

bool als_supported(int Kn, int RR) { return RR <= 256 && Kn <= 1024; }

int64_t als_chunks(const AlsGeom& g) {
  const int64_t ntiles = (g.J + kAlsTJ - 1) / kAlsTJ;
  int64_t chunks = ntiles < 512 ? ntiles : 512;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  return (ntiles + per - 1) / per;
}

__device__ __forceinline__ int64_t cyc_base(const AlsGeom& g, int64_t j) {
  int64_t base = 0;
  for (int t = g.N - 2; t >= 0; --t) {
    const int64_t d = g.cycK[t];
    base += (j % d) * g.cycStride[t];
    j /= d;
  }
  return base;
}

__global__ __launch_bounds__(kAlsThreads) void als_partial_kernel(
    const double* __restrict__ P, AlsGeom g, const double* __restrict__ Bm,
    int64_t tiles_per_chunk, double* __restrict__ part, const int* __restrict__ done) {
  if (*done) return;
  __shared__ double Bs[kAlsTJ * 256];
  __shared__ double Ps[1024 * kAlsTJ / 16];  // Kn x TJ (Kn <= 1024 -> checked on host)
  __shared__ int64_t pbase[kAlsTJ];
  const int RR = g.RR, Kn = g.Kn;
  const int nM = Kn * RR;
  const int nout = nM + RR * RR;
  const int ob = blockIdx.y * kAlsOutBlk;  // first output of this work-group's block
  // rows of P_<n> that the block's M outputs touch
  const int irow0 = min(ob, nM) / RR;
  const int irow1 = (min(ob + kAlsOutBlk, nM) + RR - 1) / RR;
  double acc[kAlsAcc];
#pragma unroll
  for (int q = 0; q < kAlsAcc; ++q) acc[q] = 0.0;
  const int64_t ntiles = (g.J + kAlsTJ - 1) / kAlsTJ;
  const int64_t t0 = (int64_t)blockIdx.x * tiles_per_chunk;
  const int64_t t1 = min(ntiles, t0 + tiles_per_chunk);
  // Kn x TJ must fit in Ps: process rows of P in slabs of kPsRows
  const int kPsRows = 1024 / 16;  // 64 rows x 16 columns
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t j0 = t * kAlsTJ;
    const int jn = (int)min((int64_t)kAlsTJ, g.J - j0);
    if (threadIdx.x < kAlsTJ) {
      const int64_t j = j0 + threadIdx.x;
      pbase[threadIdx.x] = (threadIdx.x < jn) ? cyc_base(g, j) : (int64_t)-1;
    }
    for (int x = threadIdx.x; x < kAlsTJ * RR; x += kAlsThreads) {
      const int jj = x / RR;
      Bs[x] = (jj < jn) ? Bm[(j0 + jj) * RR + (x % RR)] : 0.0;
    }
    __syncthreads();
    // Gram part (rows of P not needed)
#pragma unroll
    for (int q = 0; q < kAlsAcc; ++q) {
      const int o = ob + threadIdx.x + q * kAlsThreads;
      if (o >= nM && o < nout) {
        const int oo = o - nM;
        const int r1 = oo / RR, r2 = oo % RR;
        double sum = acc[q];
        for (int jj = 0; jj < kAlsTJ; ++jj) sum += Bs[jj * RR + r1] * Bs[jj * RR + r2];
        acc[q] = sum;
      }
    }
    // M part, slabs of rows of P_<n>
    for (int i0 = irow0; i0 < irow1; i0 += kPsRows) {
      const int rows = min(kPsRows, irow1 - i0);
      __syncthreads();
      for (int x = threadIdx.x; x < rows * kAlsTJ; x += kAlsThreads) {
        const int ii = x / kAlsTJ, jj = x % kAlsTJ;
        const int64_t pb = pbase[jj];
        Ps[x] = (pb >= 0) ? P[pb + (int64_t)(i0 + ii) * g.strideN] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kAlsAcc; ++q) {
        const int o = ob + threadIdx.x + q * kAlsThreads;
        if (o < nM) {
          const int i = o / RR, r = o % RR;
          if (i >= i0 && i < i0 + rows) {
            double sum = acc[q];
            for (int jj = 0; jj < kAlsTJ; ++jj) sum += Ps[(i - i0) * kAlsTJ + jj] * Bs[jj * RR + r];
            acc[q] = sum;
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kAlsAcc; ++q) {
    const int o = ob + threadIdx.x + q * kAlsThreads;
    if (o < nout && o < ob + kAlsOutBlk) part[(int64_t)blockIdx.x * nout + o] = acc[q];
  }
}

hipError_t launch_als_partial(const double* P, const AlsGeom& g, const double* Bm,
                              double* part, int64_t chunks, const int* done, hipStream_t s) {
  const int64_t ntiles = (g.J + kAlsTJ - 1) / kAlsTJ;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  const int nout = g.Kn * g.RR + g.RR * g.RR;
  const unsigned oblocks = (unsigned)((nout + kAlsOutBlk - 1) / kAlsOutBlk);
  prof_begin("als_partial", s);
  hipLaunchKernelGGL(als_partial_kernel, dim3((unsigned)chunks, oblocks), dim3(kAlsThreads), 0, s,
                     P, g, Bm, per, part, done);
  prof_end(s);
  return hipGetLastError();
}

__global__ void als_reduce_kernel(const double* __restrict__ part, int64_t chunks, int nout,
                                  double* __restrict__ sum, const int* __restrict__ done) {
  if (*done) return;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += part[c * nout + o];
  sum[o] = s;
}

hipError_t launch_als_reduce(const double* part, int64_t chunks, int nout, double* sum,
                             const int* done, hipStream_t s) {
  prof_begin("als_reduce", s);
  hipLaunchKernelGGL(als_reduce_kernel, dim3((nout + 255) / 256), dim3(256), 0, s, part, chunks,
                     nout, sum, done);
  prof_end(s);
  return hipGetLastError();
}

// MG = [M (Kn x RR) | Gram (RR x RR)].  Cholesky (right-looking, lower), then each thread
// solves L L^T w = m for one row m of M and writes row i of the new core.  With in_lds every
// work-group factors its own copy of the Gram in LDS and solves rows blockIdx.x,
// blockIdx.x + gridDim.x, ..; otherwise one work-group factors it in place in MG.
__global__ __launch_bounds__(256) void als_solve_kernel(double* __restrict__ MG, AlsGeom g,
                                                        double* __restrict__ Zn,
                                                        unsigned* __restrict__ status,
                                                        const int* __restrict__ done,
                                                        int in_lds) {
  if (*done) return;
  extern __shared__ double sm_g[];
  __shared__ int failed;
  const int RR = g.RR, Kn = g.Kn;
  double* M = MG;
  double* G = in_lds ? sm_g : MG + (int64_t)Kn * RR;
  if (in_lds)
    for (int x = threadIdx.x; x < RR * RR; x += blockDim.x) G[x] = MG[(int64_t)Kn * RR + x];
  if (threadIdx.x == 0) failed = 0;
  __syncthreads();
  for (int j = 0; j < RR; ++j) {
    if (threadIdx.x == 0) {
      const double d = G[j * RR + j];
      if (!(d > 0.0))
        failed = 1;
      else
        G[j * RR + j] = sqrt(d);
    }
    __syncthreads();
    if (failed) break;
    const double ljj = G[j * RR + j];
    for (int i = j + 1 + threadIdx.x; i < RR; i += blockDim.x) G[i * RR + j] /= ljj;
    __syncthreads();
    const int rem = RR - j - 1;
    for (int x = threadIdx.x; x < rem * rem; x += blockDim.x) {
      const int i = j + 1 + x / rem, k = j + 1 + x % rem;
      if (k <= i) G[i * RR + k] -= G[i * RR + j] * G[k * RR + j];
    }
    __syncthreads();
  }
  if (failed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
    return;
  }
  for (int i = blockIdx.x + gridDim.x * threadIdx.x; i < Kn; i += gridDim.x * blockDim.x) {
    double* m = M + (int64_t)i * RR;  // overwritten by the solution
    for (int r = 0; r < RR; ++r) {    // L y = m
      double s = m[r];
      for (int k = 0; k < r; ++k) s -= G[r * RR + k] * m[k];
      m[r] = s / G[r * RR + r];
    }
    for (int r = RR - 1; r >= 0; --r) {  // L^T w = y
      double s = m[r];
      for (int k = r + 1; k < RR; ++k) s -= G[k * RR + r] * m[k];
      m[r] = s / G[r * RR + r];
    }
    for (int a = 0; a < g.Ra; ++a)
      for (int b = 0; b < g.Rb; ++b) Zn[((int64_t)a * Kn + i) * g.Rb + b] = m[a * g.Rb + b];
  }
}

hipError_t launch_als_solve(double* MG, const AlsGeom& g, double* Zn, unsigned* status,
                            const int* done, hipStream_t s) {
  // Gram in LDS up to 96 KB (R_n R_{n+1} <= 110); then one work-group per 256 rows of the core
  const size_t lds = (size_t)g.RR * g.RR * sizeof(double);
  const int in_lds = lds <= 96 * 1024 ? 1 : 0;
  const unsigned grid = in_lds ? (unsigned)((g.Kn + 255) / 256) : 1u;
  if (in_lds) {
    const hipError_t e = hipFuncSetAttribute((const void*)als_solve_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  prof_begin("als_solve", s);
  hipLaunchKernelGGL(als_solve_kernel, dim3(grid), dim3(256), in_lds ? lds : 0, s, MG, g, Zn,
                     status, done, in_lds);
  prof_end(s);
  return hipGetLastError();
}

// ||P - Psi(Z)||^2 with Psi_<n>[i, j] = sum_r W[i, r] B[j, r], W = Z_{n,(2)} (the new core).
__global__ __launch_bounds__(256) void als_resid_kernel(const double* __restrict__ P, AlsGeom g,
                                                        const double* __restrict__ Bm,
                                                        const double* __restrict__ Zn,
                                                        int64_t per, double* __restrict__ part,
                                                        const int* __restrict__ done) {
  if (*done) return;
  __shared__ double red[16];
  const int RR = g.RR;
  double s = 0.0;
  const int64_t j0 = (int64_t)blockIdx.x * per;
  const int64_t j1 = min(g.J, j0 + per);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const int64_t pb = cyc_base(g, j);
    const double* brow = Bm + j * RR;
    for (int i = 0; i < g.Kn; ++i) {
      double psi = 0.0;
      for (int a = 0; a < g.Ra; ++a)
        for (int b = 0; b < g.Rb; ++b)
          psi += Zn[((int64_t)a * g.Kn + i) * g.Rb + b] * brow[a * g.Rb + b];
      const double d = P[pb + (int64_t)i * g.strideN] - psi;
      s += d * d;
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_als_resid(const double* P, const AlsGeom& g, const double* Bm,
                            const double* Zn, double* part, int64_t chunks, const int* done,
                            hipStream_t s) {
  const int64_t per = (g.J + chunks - 1) / chunks;
  prof_begin("als_resid", s);
  hipLaunchKernelGGL(als_resid_kernel, dim3((unsigned)chunks), dim3(256), 0, s, P, g, Bm, Zn,
                     per, part, done);
  prof_end(s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void als_err_kernel(const double* __restrict__ part,
                                                      int64_t chunks,
                                                      const double* __restrict__ pn2,
                                                      int sweep, double tol,
                                                      double* __restrict__ trace,
                                                      int* __restrict__ sweeps_run,
                                                      int* __restrict__ done) {
  if (*done) return;
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < chunks; c += blockDim.x) s += part[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double e = sqrt(s / pn2[0]);
    trace[sweep] = e;
    *sweeps_run = sweep + 1;
    if (tol > 0.0 && sweep >= 1 && fabs(e - trace[sweep - 1]) < tol) *done = 1;
  }
}

hipError_t launch_als_err(const double* part, int64_t chunks, const double* pn2, int sweep,
                          double tol, double* trace, int* sweeps_run, int* done,
                          hipStream_t s) {
  prof_begin("als_err", s);
  hipLaunchKernelGGL(als_err_kernel, dim3(1), dim3(256), 0, s, part, chunks, pn2, sweep, tol,
                     trace, sweeps_run, done);
  prof_end(s);
  return hipGetLastError();
}

__global__ void als_begin_kernel(int* done, int* sweeps_run) {
  *done = 0;
  *sweeps_run = 0;
}

hipError_t launch_als_begin(int* done, int* sweeps_run, hipStream_t s) {
  hipLaunchKernelGGL(als_begin_kernel, dim3(1), dim3(1), 0, s, done, sweeps_run);
  return hipGetLastError();
}

}  // namespace rtr
