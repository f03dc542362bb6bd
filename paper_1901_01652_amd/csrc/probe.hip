// HBM read-stream probe: the achievable read bandwidth of this device, measured with the
// access pattern the passes over X use (16-byte loads, one persistent grid, several loads in
// flight per lane).  It is the measured peak the X-streaming kernels are compared against,
// next to the published 8 TB/s.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;

__global__ __launch_bounds__(kProbeThreads) void read_probe_kernel(const float4* __restrict__ x,
                                                                 int64_t n4,
                                                                 double* __restrict__ part) {
  __shared__ double red[16];
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  float s = 0.f;
  for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
    float4 v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = x[i + u * stride];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n4; i += stride) {
    const float4 v = x[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  const double t = block_sum((double)s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kProbeThreads) void probe_sum_kernel(const double* part, int n,
                                                                double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kProbeThreads) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

int probe_blocks() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipGetLastError();
  return cus * 8;
}

hipError_t launch_read_probe(const void* x, int64_t bytes, double* part, double* out,
                             hipStream_t s) {
  const int blocks = probe_blocks();
  prof_begin("read_probe", s);
  hipLaunchKernelGGL(read_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s,
                     (const float4*)x, bytes / 16, part);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_sum_kernel, dim3(1), dim3(kProbeThreads), 0, s, part, blocks, out);
  return hipGetLastError();
}

}  // namespace rtr
