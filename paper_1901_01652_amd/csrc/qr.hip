// Alg. 1 step 6: economy QR of each sketch Y_n (In x K, FP64), Householder reflections
// (Golub & Van Loan, Alg. 5.2.1), then Q = H_1 ... H_K [I_K; 0] and the sign convention
// R_ii >= 0 (a column of Q is negated where the Householder diagonal is negative).
//
// One work-group per matrix.  The matrix stays in global memory (it is tiny and
// L2-resident); each wavefront owns a subset of columns while a reflector is applied.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kQrThreads = 256;
constexpr int kQrKMax = 256;

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
  qr_one(jobs.A[job], jobs.Qwork[job], jobs.In[job], jobs.K[job], jobs.Q[job]);
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

hipError_t launch_householder_qr(const QrJobs& jobs, hipStream_t s) {
  if (jobs.count <= 0) return hipSuccess;
  for (int j = 0; j < jobs.count; ++j)
    if (jobs.K[j] > kQrKMax) return hipErrorInvalidValue;
  prof_begin("householder_qr", s);
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
