// Alg. 1 step 7 read cumulatively (Eq. 3): P = X x_1 Q_1^T ... x_N Q_N^T as a chain of
// mode products, mode 1 first.  Each product maps in (A x In x B) to out (A x K x B):
// out[a, k, b] = sum_i in[a, i, b] Q[i, k].  A thread owns one (a, b) fiber, reads it once
// (coalesced along b) and keeps its K sums in registers; Q is read with uniform
// (scalar-cache) loads.
//
// The first product reads X in the requested arithmetic: FP64, FP32, or bf16 operands with
// the FP32 refinement X_hi Q_hi + X_hi Q_lo + X_lo Q_hi (X = X_hi + X_lo, Q = Q_hi + Q_lo
// split into bf16 pairs, FP32 accumulation).  Later products act on the small FP64
// intermediate.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kTtmKMax = 64;   // outputs per thread at most; larger K spreads over threads
constexpr int kTtmKLimit = 1024;

// KC: outputs k per thread; thread (p, ks) owns fiber p = (a, b) and k in [ks KC, ks KC + KC),
// so short products with few fibers still spread over enough threads.
template <int AR, typename Tin, int KC>
__device__ __forceinline__ void ttm_thread(const Tin* __restrict__ in, int64_t A, int64_t In,
                                           int64_t B, int K, const double* __restrict__ Q,
                                           double* __restrict__ out, int64_t p, int k0) {
  using Acc = typename std::conditional<AR == kF64, double, float>::type;
  const int64_t nfib = A * B;
  if (p >= nfib || k0 >= K) return;
  const int kn = K - k0 < KC ? K - k0 : KC;
  const int64_t a = p / B, b = p % B;
  const Tin* src = in + a * In * B + b;
  Acc acc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) acc[k] = 0;
  // every k < KC accumulates (columns k >= kn read column k0, always in range, and are
  // discarded at the store), so the uniform Q loads issue back to back without branches
  auto step = [&](Tin xv, int64_t i) {
    const double* q = Q + i * K + k0;
    if constexpr (AR == kBF16) {
      const float x = (float)xv;
      const float xh = bf16_round(x);
      const float xl = bf16_round(x - xh);
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const float qf = (float)q[k < kn ? k : 0];
        const float qh = bf16_round(qf);
        const float ql = bf16_round(qf - qh);
        acc[k] += xh * qh + (xh * ql + xl * qh);
      }
    } else {
      const Acc x = (Acc)xv;
#pragma unroll
      for (int k = 0; k < KC; ++k) acc[k] += x * (Acc)q[k < kn ? k : 0];
    }
  };
  // elements i = 0, 1, ... in order; each of the kAhead registers is reloaded right after its
  // element is used, kAhead elements ahead (indices clamped to the fiber), so kAhead - 1 loads
  // are in flight while an element's sums run
  constexpr int kAhead = 4;
  const int64_t last = In - 1;
  Tin xr[kAhead];
#pragma unroll
  for (int d = 0; d < kAhead; ++d) xr[d] = src[(d < last ? d : last) * B];
  int64_t i = 0;
  for (; i + kAhead <= In; i += kAhead) {
#pragma unroll
    for (int d = 0; d < kAhead; ++d) {
      step(xr[d], i + d);
      const int64_t nx = i + d + kAhead;
      xr[d] = src[(nx < last ? nx : last) * B];
    }
  }
#pragma unroll
  for (int d = 0; d < kAhead; ++d)
    if (i + d < In) step(xr[d], i + d);
  double* dst = out + a * (int64_t)K * B + b;
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (k < kn) dst[(int64_t)(k0 + k) * B] = (double)acc[k];
}

// Grid (fiber blocks, k-groups): the k-group is the block's y index, so every wavefront reads
// the same row of Q and those loads go through the scalar cache.
template <int AR, typename Tin, int KC>
__global__ __launch_bounds__(256) void ttm_kernel(const Tin* __restrict__ in, int64_t A,
                                                  int64_t In, int64_t B, int K,
                                                  const double* __restrict__ Q,
                                                  double* __restrict__ out) {
  ttm_thread<AR, Tin, KC>(in, A, In, B, K, Q, out, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                          (int)blockIdx.y * KC);
}

// One mode product for many tensors in one launch (the batched compression).
template <int AR, typename Tin, int KC>
__global__ __launch_bounds__(256) void ttm_list_kernel(const TtmJob* __restrict__ jobs,
                                                       const int64_t* __restrict__ block_start,
                                                       int njobs) {
  const int j = find_job(block_start, njobs, blockIdx.x);
  const TtmJob g = jobs[j];
  const int64_t t = ((int64_t)blockIdx.x - block_start[j]) * 256 + threadIdx.x;
  const int64_t nfib = g.A * g.B;
  ttm_thread<AR, Tin, KC>((const Tin*)g.in, g.A, g.In, g.B, g.K, g.Q, g.out, t % nfib,
                          (int)(t / nfib) * KC);
}

int64_t ttm_job_blocks(const TtmJob& g, int kc) {
  return (g.A * g.B * ((g.K + kc - 1) / kc) + 255) / 256;
}

hipError_t launch_ttm_list(Arith ar, bool first, int kc, const TtmJob* jobs,
                           const int64_t* block_start, int njobs, int64_t blocks, hipStream_t s) {
  if (njobs < 1) return hipSuccess;
  prof_begin(first ? "ttm_first" : "ttm", s);
#define RTR_TTM_LIST(KC_)                                                                      \
  if (!first || ar == kF64)                                                                    \
    hipLaunchKernelGGL((ttm_list_kernel<kF64, double, KC_>), dim3((unsigned)blocks), dim3(256), \
                       0, s, jobs, block_start, njobs);                                        \
  else if (ar == kF32)                                                                         \
    hipLaunchKernelGGL((ttm_list_kernel<kF32, float, KC_>), dim3((unsigned)blocks), dim3(256),  \
                       0, s, jobs, block_start, njobs);                                        \
  else                                                                                         \
    hipLaunchKernelGGL((ttm_list_kernel<kBF16, float, KC_>), dim3((unsigned)blocks), dim3(256), \
                       0, s, jobs, block_start, njobs);
  if (kc == 4) {
    RTR_TTM_LIST(4)
  } else if (kc == 16) {
    RTR_TTM_LIST(16)
  } else {
    RTR_TTM_LIST(64)
  }
#undef RTR_TTM_LIST
  prof_end(s);
  return hipGetLastError();
}

template <int KC>
static void launch_ttm_kc(Arith ar, bool first, const void* in, const ModeView& v, int K,
                          const double* Q, double* out, hipStream_t s) {
  const dim3 blocks((unsigned)((v.A * v.B + 255) / 256), (unsigned)((K + KC - 1) / KC));
  if (!first || ar == kF64) {
    hipLaunchKernelGGL((ttm_kernel<kF64, double, KC>), dim3(blocks), dim3(256), 0, s,
                       (const double*)in, v.A, v.In, v.B, K, Q, out);
  } else if (ar == kF32) {
    hipLaunchKernelGGL((ttm_kernel<kF32, float, KC>), dim3(blocks), dim3(256), 0, s,
                       (const float*)in, v.A, v.In, v.B, K, Q, out);
  } else {
    hipLaunchKernelGGL((ttm_kernel<kBF16, float, KC>), dim3(blocks), dim3(256), 0, s,
                       (const float*)in, v.A, v.In, v.B, K, Q, out);
  }
}

hipError_t launch_ttm(Arith ar, bool first, const void* in, const ModeView& v, int K,
                      const double* Q, double* out, hipStream_t s) {
  if (K < 1 || K > kTtmKLimit) return hipErrorInvalidValue;
  const int64_t fibers = v.A * v.B;
  prof_begin(first ? "ttm_first" : "ttm", s);
  // enough threads to cover the GPU: split K when there are few fibers
  if (fibers >= (1 << 17))
    launch_ttm_kc<kTtmKMax>(ar, first, in, v, K, Q, out, s);
  else if (fibers >= (1 << 14))
    launch_ttm_kc<4>(ar, first, in, v, K, Q, out, s);
  else
    launch_ttm_kc<1>(ar, first, in, v, K, Q, out, s);
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Sum of squares, two stages with a fixed summation order.
// ---------------------------------------------------------------------------------------
constexpr int kSsBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial_kernel(const T* __restrict__ x, int64_t n,
                                                            double* __restrict__ partial) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    s += v * v;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sum_final_kernel(const double* __restrict__ partial,
                                                        int count, double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) s += partial[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch_sum(const double* x, int64_t count, double* out, hipStream_t s) {
  prof_begin("sum", s);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, s, x, (int)count, out);
  prof_end(s);
  return hipGetLastError();
}

hipError_t launch_sumsq(bool f32, const void* x, int64_t n, double* partial, double* out,
                        hipStream_t s) {
  prof_begin("sumsq", s);
  if (f32)
    hipLaunchKernelGGL(sumsq_partial_kernel<float>, dim3(kSsBlocks), dim3(256), 0, s,
                       (const float*)x, n, partial);
  else
    hipLaunchKernelGGL(sumsq_partial_kernel<double>, dim3(kSsBlocks), dim3(256), 0, s,
                       (const double*)x, n, partial);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, s, partial, kSsBlocks, out);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
