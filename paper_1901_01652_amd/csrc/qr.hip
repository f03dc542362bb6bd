// Alg. 1 step 6: economy QR of each sketch Y_n (In x K, FP64), Householder reflections
// (Golub & Van Loan, Alg. 5.2.1), then Q = H_1 ... H_K [I_K; 0] and the sign convention
// R_ii >= 0 (a column of Q is negated where the Householder diagonal is negative).
//
// One work-group per matrix.  A matrix whose factors fit in LDS (2 In K doubles up to 150 KB)
// is factored there; a taller one with K <= 64 by TSQR (blocks of rows factored in LDS, then
// their stacked R factors, recursively); anything else stays in global memory (L2-resident),
// each wavefront owning a subset of columns while a reflector is applied.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kQrThreads = 256;
constexpr int kQrKMax = 256;
constexpr int kQrLdsThreads = 512;
constexpr size_t kQrLdsMax = 150 * 1024;

static __host__ __device__ inline size_t qr_lds_bytes(int64_t In, int K) {
  return (size_t)(2 * In * K + 3 * K) * sizeof(double);
}
static __host__ __device__ inline bool qr_fits_lds(int64_t In, int K) {
  return qr_lds_bytes(In, K) <= kQrLdsMax;
}
// Rows of one TSQR block: the most the LDS factorization takes.
static __host__ __device__ inline int64_t tsqr_block_max(int K) {
  return (int64_t)(kQrLdsMax / sizeof(double) - 3 * K) / (2 * K);
}
constexpr int kTsqrKMax = 64;
// Whether TSQR can factor a rows x K matrix with ``wcap`` doubles of scratch and the matrix's
// own ``acap`` doubles: at every level the blocks have at least K rows, the stacked factors
// (mK x K) fit the level's scratch, the next level's Q fits the front of the level's matrix
// and its scratch is the rest; the last level fits the LDS factorization.
static __host__ __device__ inline bool tsqr_ok(int64_t rows, int K, int64_t wcap, int64_t acap) {
  if (K > kTsqrKMax) return false;
  for (int level = 0; level < 32; ++level) {
    if (qr_fits_lds(rows, K)) return true;
    const int64_t m = (rows + tsqr_block_max(K) - 1) / tsqr_block_max(K);
    if (rows / m < K) return false;
    const int64_t mk = m * K;
    if (mk * K > wcap || mk * K > acap) return false;
    const int64_t w2 = acap - mk * K;
    acap = wcap;
    wcap = w2;
    rows = mk;
  }
  return false;
}
// A matrix beyond the LDS factorization that TSQR takes (with the caller's two In x K buffers).
static __host__ __device__ inline bool qr_tall(int64_t In, int K) {
  return !qr_fits_lds(In, K) && tsqr_ok(In, K, In * K, In * K);
}

// One matrix per work-group: A (column-major In x K, overwritten), Qm scratch, Qout row-major.
__device__ __forceinline__ void qr_one(double* A, double* Qm, int64_t In, int K, double* Qout) {
  __shared__ double red[16];
  __shared__ double rdiag[kQrKMax];
  __shared__ double vtv[kQrKMax];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int nw = kQrThreads / kWave;

  for (int c = 0; c < K; ++c) {
    double* a = A + (int64_t)c * In;
    double s2 = 0.0;
    for (int64_t i = c + threadIdx.x; i < In; i += kQrThreads) s2 += a[i] * a[i];
    s2 = block_sum(s2, red);
    const double alpha = a[c];
    const double nrm = sqrt(s2);
    const double beta = (alpha >= 0.0) ? -nrm : nrm;  // R_cc before the sign fix
    const double vv = 2.0 * nrm * (nrm + fabs(alpha));  // v^T v with v_c = alpha - beta
    __syncthreads();
    if (threadIdx.x == 0) {
      rdiag[c] = beta;
      vtv[c] = vv;
      a[c] = alpha - beta;
    }
    __syncthreads();
    if (vv > 0.0) {
      for (int cc = c + 1 + wid; cc < K; cc += nw) {
        double* b = A + (int64_t)cc * In;
        double d = 0.0;
        for (int64_t i = c + lane; i < In; i += kWave) d += a[i] * b[i];
        d = wave_sum(d);
        const double f = 2.0 * d / vv;
        for (int64_t i = c + lane; i < In; i += kWave) b[i] -= f * a[i];
      }
    }
    __syncthreads();
  }
  // Q = H_0 H_1 ... H_{K-1} [I; 0]; H_c only touches columns c..K-1 of the partial product.
  for (int64_t p = threadIdx.x; p < In * K; p += kQrThreads) {
    const int64_t col = p / In, row = p % In;
    Qm[p] = (row == col) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int c = K - 1; c >= 0; --c) {
    const double vv = vtv[c];
    if (vv > 0.0) {
      const double* a = A + (int64_t)c * In;
      for (int cc = c + wid; cc < K; cc += nw) {
        double* q = Qm + (int64_t)cc * In;
        double d = 0.0;
        for (int64_t i = c + lane; i < In; i += kWave) d += a[i] * q[i];
        d = wave_sum(d);
        const double f = 2.0 * d / vv;
        for (int64_t i = c + lane; i < In; i += kWave) q[i] -= f * a[i];
      }
    }
    __syncthreads();
  }
  for (int64_t p = threadIdx.x; p < In * K; p += kQrThreads) {
    const int64_t row = p / K;
    const int col = (int)(p % K);
    const double sg = (rdiag[col] < 0.0) ? -1.0 : 1.0;
    Qout[p] = sg * Qm[(int64_t)col * In + row];
  }
}

__global__ __launch_bounds__(kQrThreads) void householder_qr_kernel(QrJobs jobs) {
  const int job = blockIdx.x;
  // taken by householder_qr_lds_kernel or the TSQR launches
  if (qr_fits_lds(jobs.In[job], jobs.K[job]) || qr_tall(jobs.In[job], jobs.K[job])) return;
  qr_one(jobs.A[job], jobs.Qwork[job], jobs.In[job], jobs.K[job], jobs.Q[job]);
}

// The same factorization with the matrix and the product Q held in LDS (In x K each, column-
// major).  Wavefront w owns the columns j = w mod 8 throughout.  Step c: every wavefront forms
// the reflector of column c itself (the norm of column c from row c on, alpha, beta, v^T v:
// identical arithmetic in each), then applies it to the columns it owns (dot product, scale,
// update), one barrier per step since column c comes from its owner.  Q = H_0 .. H_{K-1} [I; 0]
// is accumulated backwards on the owners' columns of Q and needs no barrier at all: the
// reflectors are read only and every column of Q stays with one wavefront.
// Ag: In x K column-major with leading dimension lda; Qo: In x K row-major; Ro (optional): the
// K x K factor R, with the same sign convention as Q (R_ii >= 0), column-major, leading
// dimension ldr.
__device__ void qr_lds_core(const double* Ag, int64_t lda, int In, int K, double* qsm,
                            double* Qo, double* Ro, int64_t ldr) {
  double* A = qsm;                       // In x K, column-major
  double* Q = A + (size_t)In * K;        // In x K, column-major
  double* vdiag = Q + (size_t)In * K;    // v_c at row c (A keeps alpha there)
  double* rdiag = vdiag + K;             // R_cc before the sign fix
  double* vtv = rdiag + K;               // v^T v
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  constexpr int kW = kQrLdsThreads / kWave;
  for (int p = tid; p < In * K; p += kQrLdsThreads) A[p] = Ag[(int64_t)(p / In) * lda + p % In];
  for (int p = tid; p < In * K; p += kQrLdsThreads) Q[p] = (p % In == p / In) ? 1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c < K; ++c) {
    const double* a = A + (size_t)c * In;
    double s2 = 0.0;
    for (int i = c + lane; i < In; i += kWave) s2 = fma(a[i], a[i], s2);
    s2 = wave_sum(s2);
    const double alpha = a[c];
    const double nrm = sqrt(s2);
    const double beta = (alpha >= 0.0) ? -nrm : nrm;
    const double vv = 2.0 * nrm * (nrm + fabs(alpha));
    const double vc = alpha - beta;
    if (tid == 0) {
      vdiag[c] = vc;
      rdiag[c] = beta;
      vtv[c] = vv;
    }
    if (vv > 0.0) {
      for (int j = c + 1 + ((wid - (c + 1)) % kW + kW) % kW; j < K; j += kW) {
        double* b = A + (size_t)j * In;
        double d = 0.0;
        for (int i = c + 1 + lane; i < In; i += kWave) d = fma(a[i], b[i], d);
        d = wave_sum(d);
        const double f = 2.0 * fma(vc, b[c], d) / vv;
        if (lane == 0) b[c] -= f * vc;
        for (int i = c + 1 + lane; i < In; i += kWave) b[i] = fma(-f, a[i], b[i]);
      }
    }
    __syncthreads();
  }
  // Q = H_0 H_1 .. H_{K-1} [I; 0]: H_c touches rows and columns c.. of the partial product
  for (int c = K - 1; c >= 0; --c) {
    const double vv = vtv[c];
    if (!(vv > 0.0)) continue;
    const double* a = A + (size_t)c * In;
    const double vc = vdiag[c];
    for (int j = c + ((wid - c) % kW + kW) % kW; j < K; j += kW) {
      double* q = Q + (size_t)j * In;
      double d = 0.0;
      for (int i = c + 1 + lane; i < In; i += kWave) d = fma(a[i], q[i], d);
      d = wave_sum(d);
      const double f = 2.0 * fma(vc, q[c], d) / vv;
      if (lane == 0) q[c] -= f * vc;
      for (int i = c + 1 + lane; i < In; i += kWave) q[i] = fma(-f, a[i], q[i]);
    }
  }
  __syncthreads();
  for (int p = tid; p < In * K; p += kQrLdsThreads) {
    const int row = p / K, col = p % K;
    Qo[p] = (rdiag[col] < 0.0 ? -1.0 : 1.0) * Q[(size_t)col * In + row];
  }
  if (Ro)
    for (int p = tid; p < K * K; p += kQrLdsThreads) {
      const int r = p % K, c = p / K;
      const double v = r < c ? A[(size_t)c * In + r] : (r == c ? rdiag[c] : 0.0);
      Ro[(int64_t)c * ldr + r] = (rdiag[r] < 0.0 ? -1.0 : 1.0) * v;
    }
}

__global__ __launch_bounds__(kQrLdsThreads) void householder_qr_lds_kernel(QrJobs jobs) {
  const int job = blockIdx.x;
  if (!qr_fits_lds(jobs.In[job], jobs.K[job]) || qr_tall(jobs.In[job], jobs.K[job])) return;
  extern __shared__ __align__(16) double qsm[];
  qr_lds_core(jobs.A[job], jobs.In[job], (int)jobs.In[job], jobs.K[job], qsm, jobs.Q[job],
              nullptr, 0);
}

// Tall-skinny QR (TSQR): the rows in m blocks of at least 2K each, block b factored in LDS
// (Q_b into the rows of Q, R_b into rows bK..bK+K-1 of the stacked S); then S (mK x K) is
// factored the same way, recursively, and Q_b <- Q_b Q_S[bK..bK+K-1, :].  With R_ii >= 0 at
// the top the result is the unique such factor of the whole matrix.
__device__ __forceinline__ int64_t tsqr_row0(int64_t rows, int m, int b) {
  return rows * b / m;
}

__global__ __launch_bounds__(kQrLdsThreads) void qr_block_kernel(const double* A, int64_t rows,
                                                                 int K, int m, double* Q,
                                                                 double* S) {
  extern __shared__ __align__(16) double qsm[];
  const int b = blockIdx.x;
  const int64_t r0 = tsqr_row0(rows, m, b), r1 = tsqr_row0(rows, m, b + 1);
  qr_lds_core(A + r0, rows, (int)(r1 - r0), K, qsm, Q + r0 * K, S + (int64_t)b * K,
              (int64_t)m * K);
}

__global__ __launch_bounds__(64) void qr_combine_kernel(double* Q, int64_t rows, int K, int m,
                                                        const double* QS) {
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (r >= rows) return;
  int b = (int)(r * m / rows);
  while (b + 1 < m && tsqr_row0(rows, m, b + 1) <= r) ++b;
  while (b > 0 && tsqr_row0(rows, m, b) > r) --b;
  double q[kTsqrKMax];
#pragma unroll
  for (int c = 0; c < kTsqrKMax; ++c) q[c] = c < K ? Q[r * K + c] : 0.0;
  const double* T = QS + (int64_t)b * K * K;  // rows bK.. of Q_S, row-major
  for (int c2 = 0; c2 < K; ++c2) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kTsqrKMax; ++c)
      if (c < K) acc = fma(q[c], T[(int64_t)c * K + c2], acc);
    Q[r * K + c2] = acc;
  }
}

// Any number of matrices from a device job list (one work-group each).
__global__ __launch_bounds__(kQrThreads) void qr_list_kernel(const SketchJob* __restrict__ jobs,
                                                             double* const* __restrict__ work,
                                                             double* const* __restrict__ Qout) {
  const SketchJob g = jobs[blockIdx.x];
  qr_one(g.Ycol, work[blockIdx.x], g.In, g.K, Qout[blockIdx.x]);
}

hipError_t launch_qr_list(const SketchJob* jobs, double* const* work, double* const* Qout,
                          int njobs, hipStream_t s) {
  if (njobs < 1) return hipSuccess;
  prof_begin("householder_qr", s);
  hipLaunchKernelGGL(qr_list_kernel, dim3((unsigned)njobs), dim3(kQrThreads), 0, s, jobs, work, Qout);
  prof_end(s);
  return hipGetLastError();
}

// A (rows x K, column-major, acap doubles) is consumed; Q (rows x K, row-major) receives the
// factor; W (wcap doubles) is scratch.  The stacked factors of each level go to W, the next
// level's Q to the front of A (free once the block factorizations have read it), its scratch to
// the rest of A; tsqr_ok checked that every level fits.
static hipError_t tsqr(double* A, int64_t rows, int K, double* Q, double* W, int64_t wcap,
                       int64_t acap, hipStream_t s) {
  if (qr_fits_lds(rows, K)) {
    QrJobs one{};
    one.count = 1;
    one.A[0] = A;
    one.Qwork[0] = W;
    one.In[0] = rows;
    one.K[0] = K;
    one.Q[0] = Q;
    hipLaunchKernelGGL(householder_qr_lds_kernel, dim3(1), dim3(kQrLdsThreads),
                       qr_lds_bytes(rows, K), s, one);
    return hipGetLastError();
  }
  if (!tsqr_ok(rows, K, wcap, acap)) return hipErrorInvalidValue;
  const int m = (int)((rows + tsqr_block_max(K) - 1) / tsqr_block_max(K));
  const int64_t blk = (rows + m - 1) / m;  // the largest block
  hipLaunchKernelGGL(qr_block_kernel, dim3(m), dim3(kQrLdsThreads), qr_lds_bytes(blk, K), s, A,
                     rows, K, m, Q, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mk = (int64_t)m * K;
  if ((e = tsqr(W, mk, K, A, A + mk * K, acap - mk * K, wcap, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(qr_combine_kernel, dim3((unsigned)((rows + 63) / 64)), dim3(64), 0, s, Q, rows,
                     K, m, (const double*)A);
  return hipGetLastError();
}

hipError_t launch_householder_qr(const QrJobs& jobs, hipStream_t s) {
  if (jobs.count <= 0) return hipSuccess;
  for (int j = 0; j < jobs.count; ++j)
    if (jobs.K[j] > kQrKMax) return hipErrorInvalidValue;
  size_t lds = 0;
  bool any_global = false;
  for (int j = 0; j < jobs.count; ++j) {
    if (qr_fits_lds(jobs.In[j], jobs.K[j]))
      lds = std::max(lds, qr_lds_bytes(jobs.In[j], jobs.K[j]));
    else if (!qr_tall(jobs.In[j], jobs.K[j]))
      any_global = true;
  }
  prof_begin("householder_qr", s);
  hipError_t e = hipFuncSetAttribute((const void*)householder_qr_lds_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQrLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)qr_block_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kQrLdsMax);
  if (e != hipSuccess) return e;
  if (lds > 0)
    hipLaunchKernelGGL(householder_qr_lds_kernel, dim3(jobs.count), dim3(kQrLdsThreads), lds, s,
                       jobs);
  for (int j = 0; j < jobs.count; ++j)
    if (qr_tall(jobs.In[j], jobs.K[j]) &&
        (e = tsqr(jobs.A[j], jobs.In[j], jobs.K[j], jobs.Q[j], jobs.Qwork[j],
                  jobs.In[j] * jobs.K[j], jobs.In[j] * jobs.K[j], s)) != hipSuccess)
      return e;
  if (any_global)
    hipLaunchKernelGGL(householder_qr_kernel, dim3(jobs.count), dim3(kQrThreads), 0, s, jobs);
  prof_end(s);
  return hipGetLastError();
}

__global__ void identity_kernel(double* Q, int64_t In) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < In * In) Q[p] = (p / In == p % In) ? 1.0 : 0.0;
}

hipError_t launch_identity(double* Q, int64_t In, hipStream_t s) {
  const unsigned blocks = (unsigned)((In * In + 255) / 256);
  prof_begin("identity", s);
  hipLaunchKernelGGL(identity_kernel, dim3(blocks), dim3(256), 0, s, Q, In);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
