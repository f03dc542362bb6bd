// Alg. 1 steps 4-5: Y_n = X_(n) M_n with the Gaussian M_n generated on the fly, and the
// fiber form of the power step Y'_n = X_(n) (X_(n)^T Q_n).
//
// General kernels for any order and size.  X is viewed for mode n as A x In x B; column j
// of X_(n) is (a, b) with j = a*B + b, which is the row-major index of the other modes, so
// row j of M_n is stream elements j*K .. j*K+K-1.  A work-group owns a chunk of column
// tiles and a block of 64 rows; it draws the tile's rows of M_n once into LDS, stages the
// X tile in LDS and accumulates its rows of the partial sketch in registers.  Partials
// are summed in a fixed order by reduce_partials (deterministic, no atomics).
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

template <int AR>
struct Ar;
template <>
struct Ar<kF64> {
  using X = double;
  using Acc = double;
  static __device__ __forceinline__ double in(double v) { return v; }
  static __device__ __forceinline__ double rnd(double v) { return v; }
};
template <>
struct Ar<kF32> {
  using X = float;
  using Acc = float;
  static __device__ __forceinline__ float in(float v) { return v; }
  static __device__ __forceinline__ float rnd(float v) { return v; }
};
template <>
struct Ar<kBF16> {  // bf16 operands, exact products, FP32 accumulation
  using X = float;
  using Acc = float;
  static __device__ __forceinline__ float in(float v) { return bf16_round(v); }
  static __device__ __forceinline__ float rnd(float v) { return bf16_round(v); }
};

constexpr int kSkTI = 64;   // rows per block
constexpr int kSkTJ = 32;   // columns per tile
constexpr int kSkKMax = 64; // projection size limit of the general kernel
constexpr int kSkThreads = 256;

// One work-group's share of a sketch: column tiles [t0, t1) of X_(n), rows [i0, i0 + 64),
// accumulated into out[(i) * K + k] (this work-group's partial record, In x K).
template <int AR>
__device__ __forceinline__ void sketch_range(const typename Ar<AR>::X* __restrict__ X, int64_t A,
                                             int64_t In, int64_t B, int K, uint64_t seed,
                                             uint32_t stream, uint32_t tid, int64_t t0, int64_t t1,
                                             int64_t i0, typename Ar<AR>::Acc* __restrict__ out,
                                             const KrArgs& kr) {
  using Acc = typename Ar<AR>::Acc;
  __shared__ Acc Xs[kSkTI][kSkTJ + 1];
  __shared__ Acc Om[kSkTJ * kSkKMax];
  __shared__ int64_t colbase[kSkTJ];
  const int64_t J = A * B;
  const int il = threadIdx.x % kSkTI;
  const int kg = threadIdx.x / kSkTI;  // 4 groups of columns k = kg + 4q
  Acc acc[kSkKMax / 4];
#pragma unroll
  for (int q = 0; q < kSkKMax / 4; ++q) acc[q] = 0;

  for (int64_t t = t0; t < t1; ++t) {
    const int64_t j0 = t * kSkTJ;
    const int64_t jn = min((int64_t)kSkTJ, J - j0);
    const int64_t e0 = j0 * K, e1 = (j0 + jn) * K;
    if (kr.f) {  // Khatri-Rao test matrix: products of the other modes' factor rows
      const Acc* F = (const Acc*)kr.f;
      for (int x = threadIdx.x; x < jn * K; x += kSkThreads) {
        const int jj = x / K, k = x % K;
        int64_t r = j0 + jj;
        int64_t row[7];
#pragma unroll
        for (int m = 6; m >= 0; --m) {
          if (m < kr.nm) {
            const int d = kr.dim[m];
            row[m] = kr.off[m] + (r % d) * kr.ld;
            r /= d;
          }
        }
        Acc v = 1;
#pragma unroll
        for (int m = 0; m < 7; ++m)
          if (m < kr.nm) v *= F[row[m] + k];
        Om[x] = Ar<AR>::rnd(v);
      }
    } else {
      for (int64_t c = (e0 >> 2) + threadIdx.x; c <= ((e1 - 1) >> 2); c += kSkThreads) {
        Acc z[4];
        normals4(seed, stream, tid, (uint64_t)c, z);
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const int64_t e = 4 * c + l;
          if (e >= e0 && e < e1) Om[e - e0] = Ar<AR>::rnd(z[l]);
        }
      }
    }
    for (int x = (int)(jn * K) + threadIdx.x; x < kSkTJ * K; x += kSkThreads) Om[x] = 0;
    if (threadIdx.x < kSkTJ) {
      const int64_t j = j0 + threadIdx.x;
      colbase[threadIdx.x] = (j < J) ? (j / B) * In * B + (j % B) : (int64_t)-1;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < kSkTI * kSkTJ; l += kSkThreads) {
      int ii, jj;
      if (B >= kSkTJ) {
        jj = l % kSkTJ;
        ii = l / kSkTJ;
      } else {
        ii = l % kSkTI;
        jj = l / kSkTI;
      }
      const int64_t i = i0 + ii;
      const int64_t cb = colbase[jj];
      Acc v = 0;
      if (i < In && cb >= 0) v = Ar<AR>::in(X[cb + i * B]);
      Xs[ii][jj] = v;
    }
    __syncthreads();
    for (int jj = 0; jj < kSkTJ; ++jj) {
      const Acc x = Xs[il][jj];
#pragma unroll
      for (int q = 0; q < kSkKMax / 4; ++q) {
        const int k = kg + 4 * q;
        if (k < K) acc[q] += x * Om[jj * K + k];
      }
    }
    __syncthreads();
  }
  const int64_t i = i0 + il;
  if (i < In) {
#pragma unroll
    for (int q = 0; q < kSkKMax / 4; ++q) {
      const int k = kg + 4 * q;
      if (k < K) out[i * K + k] = acc[q];
    }
  }
}

template <int AR>
__global__ __launch_bounds__(kSkThreads) void sketch_partial_kernel(
    const typename Ar<AR>::X* __restrict__ X, int64_t A, int64_t In, int64_t B, int K,
    uint64_t seed, uint32_t stream, uint32_t tid, int64_t ntiles, int64_t tiles_per_chunk,
    typename Ar<AR>::Acc* __restrict__ partial, KrArgs kr) {
  const int64_t chunk = blockIdx.x;
  const int64_t t0 = chunk * tiles_per_chunk;
  const int64_t t1 = min(ntiles, t0 + tiles_per_chunk);
  sketch_range<AR>(X, A, In, B, K, seed, stream, tid, t0, t1, (int64_t)blockIdx.y * kSkTI,
                   partial + chunk * In * K, kr);
}

int64_t sketch_chunks(const ModeView& v, int K) {
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + kSkTJ - 1) / kSkTJ;
  const int64_t nrb = (v.In + kSkTI - 1) / kSkTI;
  int64_t target = 2048 / nrb;
  if (target < 1) target = 1;
  int64_t chunks = ntiles < target ? ntiles : target;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  return (ntiles + per - 1) / per;
}

hipError_t launch_sketch_partial(Arith ar, const void* X, const ModeView& v, int K,
                                 uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                                 void* partial, int64_t chunks, hipStream_t s, const KrArgs* kr) {
  if (K > kSkKMax) return hipErrorInvalidValue;
  KrArgs ka{};
  if (kr) ka = *kr;
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + kSkTJ - 1) / kSkTJ;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  const int64_t nrb = (v.In + kSkTI - 1) / kSkTI;
  dim3 grid((unsigned)chunks, (unsigned)nrb);
  prof_begin("sketch_partial", s);
  switch (ar) {
    case kF64:
      hipLaunchKernelGGL(sketch_partial_kernel<kF64>, grid, dim3(kSkThreads), 0, s,
                         (const double*)X, v.A, v.In, v.B, K, seed, stream_word, tensor_id,
                         ntiles, per, (double*)partial, ka);
      break;
    case kF32:
      hipLaunchKernelGGL(sketch_partial_kernel<kF32>, grid, dim3(kSkThreads), 0, s,
                         (const float*)X, v.A, v.In, v.B, K, seed, stream_word, tensor_id,
                         ntiles, per, (float*)partial, ka);
      break;
    default:
      hipLaunchKernelGGL(sketch_partial_kernel<kBF16>, grid, dim3(kSkThreads), 0, s,
                         (const float*)X, v.A, v.In, v.B, K, seed, stream_word, tensor_id,
                         ntiles, per, (float*)partial, ka);
  }
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void normals_kernel(uint64_t seed, uint32_t stream,
                                                      uint32_t tid, int64_t start,
                                                      int64_t count, T* __restrict__ out) {
  const int64_t c = (start >> 2) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * c >= start + count) return;
  T z[4];
  normals4(seed, stream, tid, (uint64_t)c, z);
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int64_t e = 4 * c + l;
    if (e >= start && e < start + count) out[e - start] = z[l];
  }
}

hipError_t launch_normals(bool f32, uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                          int64_t start, int64_t count, void* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t calls = ((start + count - 1) >> 2) - (start >> 2) + 1;
  const unsigned blocks = (unsigned)((calls + 255) / 256);
  prof_begin("normals", s);
  if (f32)
    hipLaunchKernelGGL(normals_kernel<float>, dim3(blocks), dim3(256), 0, s, seed, stream_word,
                       tensor_id, start, count, (float*)out);
  else
    hipLaunchKernelGGL(normals_kernel<double>, dim3(blocks), dim3(256), 0, s, seed, stream_word,
                       tensor_id, start, count, (double*)out);
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Power step, fiber form: for each column x_j of X_(n), w_j = Q^T x_j, Y' += x_j w_j^T.
// The work-group keeps Q and a full-height X tile (In x TJ) in LDS.
// ---------------------------------------------------------------------------------------
constexpr int kPwAccMax = 32;          // outputs per thread: In*K <= 256*32
constexpr int kPwLds = 60 * 1024;      // LDS budget in bytes

template <typename Acc>
static int power_tj(int64_t In, int K) {
  const int64_t avail = kPwLds / (int64_t)sizeof(Acc) - In * K - 64;
  if (avail <= 0) return 0;
  int64_t tj = avail / (In + K + 1);
  if (tj > 64) tj = 64;
  return (int)tj;
}

template <int AR>
__global__ __launch_bounds__(kSkThreads) void power_partial_kernel(
    const typename Ar<AR>::X* __restrict__ X, int64_t A, int64_t In, int64_t B, int K,
    const double* __restrict__ Q, int TJ, int64_t ntiles, int64_t tiles_per_chunk,
    typename Ar<AR>::Acc* __restrict__ partial) {
  using Acc = typename Ar<AR>::Acc;
  extern __shared__ __align__(16) unsigned char smem[];
  int64_t* colbase = (int64_t*)smem;                    // 64 entries
  Acc* Qs = (Acc*)(smem + 64 * sizeof(int64_t));         // In x K
  Acc* Xs = Qs + In * K;                                 // In x TJ
  Acc* Ws = Xs + In * TJ;                                // TJ x K
  const int64_t J = A * B;
  const int64_t nout = In * K;
  for (int64_t p = threadIdx.x; p < nout; p += kSkThreads) Qs[p] = Ar<AR>::rnd((Acc)Q[p]);
  Acc acc[kPwAccMax];
#pragma unroll
  for (int q = 0; q < kPwAccMax; ++q) acc[q] = 0;
  const int64_t t0 = (int64_t)blockIdx.x * tiles_per_chunk;
  const int64_t t1 = min(ntiles, t0 + tiles_per_chunk);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t j0 = t * TJ;
    if (threadIdx.x < TJ) {
      const int64_t j = j0 + threadIdx.x;
      colbase[threadIdx.x] = (j < J) ? (j / B) * In * B + (j % B) : (int64_t)-1;
    }
    __syncthreads();
    for (int64_t l = threadIdx.x; l < In * TJ; l += kSkThreads) {
      int64_t ii, jj;
      if (B >= TJ) {
        jj = l % TJ;
        ii = l / TJ;
      } else {
        ii = l % In;
        jj = l / In;
      }
      const int64_t cb = colbase[jj];
      Xs[ii * TJ + jj] = (cb >= 0) ? Ar<AR>::in(X[cb + ii * B]) : (Acc)0;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < TJ * K; p += kSkThreads) {
      const int jj = p / K, k = p % K;
      Acc sum = 0;
      for (int64_t i = 0; i < In; ++i) sum += Xs[i * TJ + jj] * Qs[i * K + k];
      Ws[p] = Ar<AR>::rnd(sum);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPwAccMax; ++q) {
      const int64_t o = threadIdx.x + (int64_t)q * kSkThreads;
      if (o < nout) {
        const int64_t i = o / K;
        const int k = (int)(o % K);
        Acc sum = acc[q];
        for (int jj = 0; jj < TJ; ++jj) sum += Xs[i * TJ + jj] * Ws[jj * K + k];
        acc[q] = sum;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPwAccMax; ++q) {
    const int64_t o = threadIdx.x + (int64_t)q * kSkThreads;
    if (o < nout) partial[(int64_t)blockIdx.x * nout + o] = acc[q];
  }
}

bool power_supported(Arith ar, const ModeView& v, int K) {
  if (v.In * K > (int64_t)kSkThreads * kPwAccMax) return false;
  const int tj = (ar == kF64) ? power_tj<double>(v.In, K) : power_tj<float>(v.In, K);
  return tj >= 1;
}

int64_t power_chunks(Arith ar, const ModeView& v, int K) {
  const int tj = (ar == kF64) ? power_tj<double>(v.In, K) : power_tj<float>(v.In, K);
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + tj - 1) / tj;
  int64_t chunks = ntiles < 2048 ? ntiles : 2048;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  return (ntiles + per - 1) / per;
}

hipError_t launch_power_partial(Arith ar, const void* X, const ModeView& v, int K,
                                const double* Q, void* partial, int64_t chunks,
                                hipStream_t s) {
  const bool f64 = (ar == kF64);
  const int tj = f64 ? power_tj<double>(v.In, K) : power_tj<float>(v.In, K);
  if (tj < 1) return hipErrorInvalidValue;
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + tj - 1) / tj;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  const size_t es = f64 ? sizeof(double) : sizeof(float);
  const size_t lds = 64 * sizeof(int64_t) + es * (size_t)(v.In * K + v.In * tj + tj * K);
  prof_begin("power_partial", s);
  switch (ar) {
    case kF64:
      hipLaunchKernelGGL(power_partial_kernel<kF64>, dim3((unsigned)chunks), dim3(kSkThreads),
                         lds, s, (const double*)X, v.A, v.In, v.B, K, Q, tj, ntiles, per,
                         (double*)partial);
      break;
    case kF32:
      hipLaunchKernelGGL(power_partial_kernel<kF32>, dim3((unsigned)chunks), dim3(kSkThreads),
                         lds, s, (const float*)X, v.A, v.In, v.B, K, Q, tj, ntiles, per,
                         (float*)partial);
      break;
    default:
      hipLaunchKernelGGL(power_partial_kernel<kBF16>, dim3((unsigned)chunks),
                         dim3(kSkThreads), lds, s, (const float*)X, v.A, v.In, v.B, K, Q, tj,
                         ntiles, per, (float*)partial);
  }
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Y[:, k] = sum over chunks of the per-work-group partials.  A work-group of 1024 threads
// owns 64 consecutive outputs; its 16 wavefronts take every 16th chunk each (coalesced
// along the outputs), and the 16 slice sums are added in a fixed order.
template <typename P>
__device__ __forceinline__ void reduce_block(const P* __restrict__ partial, int64_t chunks,
                                             int64_t In, int K, double* __restrict__ Ycol,
                                             int64_t ldy, int64_t oblock) {
  __shared__ double part[16][65];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int64_t nout = In * K;
  const int64_t o = oblock * 64 + lane;
  double s = 0.0;
  if (o < nout) {
    // chunks slice, slice + 16, ... added in that order; four loads issued before their adds
    int64_t c = slice;
    for (; c + 48 < chunks; c += 64) {
      const double v0 = (double)partial[c * nout + o];
      const double v1 = (double)partial[(c + 16) * nout + o];
      const double v2 = (double)partial[(c + 32) * nout + o];
      const double v3 = (double)partial[(c + 48) * nout + o];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; c < chunks; c += 16) s += (double)partial[c * nout + o];
  }
  part[slice][lane] = s;
  __syncthreads();
  if (slice == 0 && o < nout) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += part[q][lane];
    const int64_t i = o / K;
    const int k = (int)(o % K);
    Ycol[(int64_t)k * ldy + i] = t;
  }
}

template <typename P>
__global__ __launch_bounds__(1024) void reduce_partials_kernel(const P* __restrict__ partial,
                                                               int64_t chunks, int64_t In, int K,
                                                               double* __restrict__ Ycol,
                                                               int64_t ldy) {
  reduce_block<P>(partial, chunks, In, K, Ycol, ldy, blockIdx.x);
}

hipError_t launch_reduce_partials(Arith ar, const void* partial, int64_t chunks, int64_t In,
                                  int K, double* Ycol, hipStream_t s, int64_t ldy) {
  if (ldy == 0) ldy = In;
  const int64_t nout = In * K;
  const unsigned blocks = (unsigned)((nout + 63) / 64);
  prof_begin("reduce_partials", s);
  if (ar == kF64)
    hipLaunchKernelGGL(reduce_partials_kernel<double>, dim3(blocks), dim3(1024), 0, s,
                       (const double*)partial, chunks, In, K, Ycol, ldy);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<float>, dim3(blocks), dim3(1024), 0, s,
                       (const float*)partial, chunks, In, K, Ycol, ldy);
  prof_end(s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Work lists for many tensors at once (the batched workload): one launch sketches every
// (tensor, mode) job, one launch sums every job's partials.  Job j owns blocks
// [block_start[j], block_start[j + 1]) of the grid; a block finds its job by binary search.
template <int AR>
__global__ __launch_bounds__(kSkThreads) void sketch_list_kernel(const SketchJob* __restrict__ jobs,
                                                                 const int64_t* __restrict__ block_start,
                                                                 int njobs) {
  const int j = find_job(block_start, njobs, blockIdx.x);
  const SketchJob g = jobs[j];
  const int64_t local = (int64_t)blockIdx.x - block_start[j];
  const int64_t chunk = local / g.nrb, rb = local % g.nrb;
  const int64_t t0 = chunk * g.per;
  const int64_t t1 = min(g.ntiles, t0 + g.per);
  KrArgs none{};
  sketch_range<AR>((const typename Ar<AR>::X*)g.X, g.A, g.In, g.B, g.K, g.seed, g.stream,
                   g.tensor_id, t0, t1, rb * kSkTI,
                   (typename Ar<AR>::Acc*)g.partial + chunk * g.In * g.K, none);
}

__global__ __launch_bounds__(1024) void reduce_list_kernel(const SketchJob* __restrict__ jobs) {
  const SketchJob g = jobs[blockIdx.y];
  if ((int64_t)blockIdx.x * 64 >= g.In * g.K) return;
  reduce_block<float>((const float*)g.partial, g.chunks, g.In, g.K, g.Ycol, g.In, blockIdx.x);
}

int64_t sketch_job_chunks(const ModeView& v, int K, int target) {
  const int64_t J = v.A * v.B;
  const int64_t ntiles = (J + kSkTJ - 1) / kSkTJ;
  int64_t chunks = ntiles < target ? ntiles : target;
  if (chunks < 1) chunks = 1;
  const int64_t per = (ntiles + chunks - 1) / chunks;
  return (ntiles + per - 1) / per;
}

void sketch_job_fill(SketchJob& g, const void* X, const ModeView& v, int K, uint64_t seed,
                     uint32_t stream_word, uint32_t tensor_id, int64_t chunks, void* partial,
                     double* Ycol) {
  g.X = X;
  g.A = v.A;
  g.In = v.In;
  g.B = v.B;
  g.K = K;
  g.seed = seed;
  g.stream = stream_word;
  g.tensor_id = tensor_id;
  g.ntiles = (v.A * v.B + kSkTJ - 1) / kSkTJ;
  g.per = (g.ntiles + chunks - 1) / chunks;
  g.chunks = chunks;
  g.nrb = (int)((v.In + kSkTI - 1) / kSkTI);
  g.partial = partial;
  g.Ycol = Ycol;
}

int64_t sketch_job_blocks(const SketchJob& g) { return g.chunks * g.nrb; }

hipError_t launch_sketch_list(Arith ar, const SketchJob* jobs, const int64_t* block_start,
                              int njobs, int64_t blocks, int64_t max_out, hipStream_t s) {
  if (njobs < 1) return hipSuccess;
  prof_begin("sketch_list", s);
  if (ar == kBF16)
    hipLaunchKernelGGL(sketch_list_kernel<kBF16>, dim3((unsigned)blocks), dim3(kSkThreads), 0, s,
                       jobs, block_start, njobs);
  else
    hipLaunchKernelGGL(sketch_list_kernel<kF32>, dim3((unsigned)blocks), dim3(kSkThreads), 0, s,
                       jobs, block_start, njobs);
  hipLaunchKernelGGL(reduce_list_kernel, dim3((unsigned)((max_out + 63) / 64), (unsigned)njobs),
                     dim3(1024), 0, s, jobs);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rtr
