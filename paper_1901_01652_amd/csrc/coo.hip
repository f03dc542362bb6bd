// Alg. 1 steps 4-5 and 7 for a tensor given by its nonzeros (coordinate list, FP64 arithmetic):
//   Y_n[i_n, :] += v M_n[j_n, :]              for every nonzero (i_1..i_N, v) and every mode n
//   P[k_1..k_N] = sum over nonzeros v Q_1[i_1, k_1] .. Q_N[i_N, k_N]
// where j_n is the column of X_(n) holding the nonzero (the other modes' indices, row-major,
// first other mode slowest) and M_n[j, k] is element j K_n + k of mode n's Gaussian stream, the
// same test matrix the dense path draws.  A nonzero whose coordinates fall outside the tensor
// is skipped and sets RTR_STATUS_INDEX_RANGE.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"

namespace rtr {

constexpr int kCooThreads = 256;

__device__ __forceinline__ bool coo_load(const CooArgs& a, int64_t z, int64_t (&i)[8], double& v) {
  bool ok = true;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    if (m < a.N) {
      i[m] = a.idx[z * a.N + m];
      ok = ok && i[m] >= 0 && i[m] < a.dims[m];
    }
  }
  v = a.f32 ? (double)((const float*)a.val)[z] : ((const double*)a.val)[z];
  return ok;
}

// One thread per (nonzero, mode): the row of M_n it needs is drawn by the Philox calls that
// cover stream elements [j K, j K + K), and v times it is added to row i_n of Y_n (FP64
// atomics: the order of the additions is not fixed, so results agree to rounding).
__global__ __launch_bounds__(kCooThreads) void coo_sketch_kernel(CooArgs a) {
  const int64_t items = a.nnz * a.N;
  for (int64_t t = (int64_t)blockIdx.x * kCooThreads + threadIdx.x; t < items;
       t += (int64_t)gridDim.x * kCooThreads) {
    const int64_t z = t / a.N;
    const int n = (int)(t - z * a.N);
    const int K = a.K[n];
    if (K == 0) continue;  // mode kept: Q_n = I
    int64_t i[8];
    double v;
    if (!coo_load(a, z, i, v)) {
      if (n == 0) atomicOr(a.status, (unsigned)RTR_STATUS_INDEX_RANGE);
      continue;
    }
    int64_t j = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m)
      if (m < a.N && m != n) j = j * a.dims[m] + i[m];
    const int64_t e0 = j * K, e1 = e0 + K;
    double* y = a.Y[n] + i[n];
    const int64_t ldY = a.dims[n];
    for (int64_t c = e0 >> 2; 4 * c < e1; ++c) {
      double r[4];
      normals4(a.seed, omega_stream(n), a.tid, (uint64_t)c, r);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int64_t e = 4 * c + l;
        if (e >= e0 && e < e1) unsafeAtomicAdd(y + (e - e0) * ldY, v * r[l]);
      }
    }
  }
}

// P as an F x B matrix (front modes 0..split-1 as rows, the rest as columns, both row-major)
// equals A B^T summed over the nonzeros with A[:, z] = v (x)_{front} Q_n[i_n, :] and
// B[:, z] = (x)_{back} Q_n[i_n, :].  Work-group (rt, ct, s) forms the 64 x 64 tile (rt, ct) over
// its slice s of the nonzeros on the FP64 matrix cores (four nonzeros per 16x16x4 product,
// wavefront w the 32 x 32 quarter w) and writes it to part[s]; coo_reduce_kernel sums the
// slices in order.
__global__ __launch_bounds__(kCooThreads) void coo_compress_kernel(CooArgs a, CooGemm g) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + (wid >> 1) * 32;
  const int64_t col0 = (int64_t)blockIdx.y * 64 + (wid & 1) * 32;
  // this lane's two operand rows and two operand columns, as per-mode offsets k_n (or -1)
  int krow[2][8], kcol[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int64_t r = row0 + 16 * h + r16, c = col0 + 16 * h + r16;
    const bool rok = r < g.F, cok = c < g.B;
#pragma unroll
    for (int m = 7; m >= 0; --m) {
      krow[h][m] = -1;
      kcol[h][m] = -1;
      if (m < g.split) {
        krow[h][m] = rok ? (int)(r % g.Kp[m]) : -1;
        r /= g.Kp[m];
      } else if (m < a.N) {
        kcol[h][m] = cok ? (int)(c % g.Kp[m]) : -1;
        c /= g.Kp[m];
      }
    }
  }
  f64x4 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t z0 = (int64_t)blockIdx.z * g.chunk;
  const int64_t z1 = min(a.nnz, z0 + g.chunk);
  for (int64_t zb = z0; zb < z1; zb += 4) {
    const int64_t z = zb + g4;
    int64_t i[8] = {};
    double v = 0.0;
    bool ok = false;
    if (z < z1) ok = coo_load(a, z, i, v);
    double av[2], bv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double x = ok ? v : 0.0, y = ok ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        if (m < g.split) {
          x = krow[h][m] < 0 ? 0.0 : x * (ok ? g.Q[m][i[m] * g.Kp[m] + krow[h][m]] : 0.0);
        } else if (m < a.N) {
          y = kcol[h][m] < 0 ? 0.0 : y * (ok ? g.Q[m][i[m] * g.Kp[m] + kcol[h][m]] : 0.0);
        }
      }
      av[h] = x;
      bv[h] = y;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) acc[p][q] = mma_f64(av[p], bv[q], acc[p][q]);
  }
  double* out = g.part + (int64_t)blockIdx.z * g.F * g.B;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = row0 + 16 * p + 4 * e + g4, c = col0 + 16 * q + r16;
        if (r < g.F && c < g.B) out[r * g.B + c] = acc[p][q][e];
      }
}

__global__ __launch_bounds__(kCooThreads) void coo_reduce_kernel(const double* part, int64_t slices,
                                                                 int64_t n, double* P) {
  for (int64_t e = (int64_t)blockIdx.x * kCooThreads + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * kCooThreads) {
    double s = 0.0;
    for (int64_t q = 0; q < slices; ++q) s += part[q * n + e];
    P[e] = s;
  }
}

__global__ __launch_bounds__(kCooThreads) void fill_kernel(double* x, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * kCooThreads + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * kCooThreads)
    x[e] = v;
}

// n doubles set to v by a kernel (not a memset node, so it may sit in a captured graph).
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + kCooThreads - 1) / kCooThreads, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(kCooThreads), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_coo_sketch(const CooArgs& a, hipStream_t s) {
  const int64_t items = a.nnz * a.N;
  if (items == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((items + kCooThreads - 1) / kCooThreads, 65536);
  prof_begin("sketch_coo", s);
  hipLaunchKernelGGL(coo_sketch_kernel, dim3((unsigned)blocks), dim3(kCooThreads), 0, s, a);
  prof_end(s);
  return hipGetLastError();
}

// Slices of the nonzeros for the compression: enough work-groups to fill the chip (about 2048
// with the output tiles), at least 64 nonzeros each, and part[] within ``max_part`` doubles.
int64_t coo_slices(int64_t nnz, int64_t F, int64_t B, int64_t max_part) {
  const int64_t tiles = ((F + 63) / 64) * ((B + 63) / 64);
  int64_t s = std::max<int64_t>(1, 2048 / tiles);
  s = std::min(s, std::max<int64_t>(1, (nnz + 63) / 64));
  s = std::min(s, std::max<int64_t>(1, max_part / (F * B)));
  return s;
}

hipError_t launch_coo_compress(const CooArgs& a, CooGemm g, double* P, hipStream_t s) {
  const int64_t n = g.F * g.B;
  prof_begin("compress_coo", s);
  if (a.nnz > 0) {
    g.chunk = ((a.nnz + g.slices - 1) / g.slices + 3) / 4 * 4;
    dim3 grid((unsigned)((g.F + 63) / 64), (unsigned)((g.B + 63) / 64), (unsigned)g.slices);
    hipLaunchKernelGGL(coo_compress_kernel, grid, dim3(kCooThreads), 0, s, a, g);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  const int64_t blocks = std::min<int64_t>((n + kCooThreads - 1) / kCooThreads, 4096);
  hipLaunchKernelGGL(coo_reduce_kernel, dim3((unsigned)blocks), dim3(kCooThreads), 0, s, g.part,
                     a.nnz > 0 ? g.slices : 0, n, P);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
