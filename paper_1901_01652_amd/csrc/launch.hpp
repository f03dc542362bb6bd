// Host-side launchers of the gfx950 kernels (one translation unit per kernel family; the
// C ABI in runtime.hip calls only these).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtr {

enum Arith { kF64 = 0, kF32 = 1, kBF16 = 2 };

// Stream word of the Gaussian test matrix of mode n (tag 1 in bits 24..31).
__host__ __device__ inline uint32_t omega_stream(int n) {
  return (1u << 24) | ((uint32_t)(n & 0xFF) << 16);
}

// X viewed for mode n as A x In x B (A = prod_{m<n} I_m, B = prod_{m>n} I_m).
struct ModeView {
  int64_t A, In, B;
};

struct Launch {
  hipStream_t stream;
  const char* name;
};
// Records launch timing when profiling is enabled (runtime.hip).
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);

// ---- sketch.hip -----------------------------------------------------------------------
// Partial sketches of one mode: partial[c][i][k] (FP64 for kF64, FP32 otherwise).
int64_t sketch_chunks(const ModeView& v, int K);
hipError_t launch_sketch_partial(Arith ar, const void* X, const ModeView& v, int K,
                                 uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                                 void* partial, int64_t chunks, hipStream_t s);
// Elements [start, start+count) of a Gaussian stream (FP64 or FP32 Box-Muller).
hipError_t launch_normals(bool f32, uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                          int64_t start, int64_t count, void* out, hipStream_t s);
// Fiber-form power step Y' = X_(n) (X_(n)^T Q), Q row-major In x K (FP64).
bool power_supported(Arith ar, const ModeView& v, int K);
int64_t power_chunks(Arith ar, const ModeView& v, int K);
hipError_t launch_power_partial(Arith ar, const void* X, const ModeView& v, int K,
                                const double* Q, void* partial, int64_t chunks,
                                hipStream_t s);
// Fixed-order sum of partials into column-major Ycol (K x In storage, Ycol[k*In+i]).
hipError_t launch_reduce_partials(Arith ar, const void* partial, int64_t chunks, int64_t In,
                                  int K, double* Ycol, hipStream_t s);

// ---- qr.hip ---------------------------------------------------------------------------
struct QrJobs {
  int count;
  double* A[8];      // column-major In x K, overwritten
  double* Qwork[8];  // column-major In x K scratch
  int64_t In[8];
  int K[8];
  double* Q[8];      // row-major In x K output
};
hipError_t launch_householder_qr(const QrJobs& jobs, hipStream_t s);
// Q = identity (In x In, row-major)
hipError_t launch_identity(double* Q, int64_t In, hipStream_t s);

// ---- compress.hip ---------------------------------------------------------------------
// out (A x K x B, FP64) = in (A x In x B) x_2 Q^T, Q row-major In x K FP64.
// ``first`` selects the input type: X (F64/F32/BF16-with-refinement) or FP64.
hipError_t launch_ttm(Arith ar, bool first, const void* in, const ModeView& v, int K,
                      const double* Q, double* out, hipStream_t s);
// Sum of squares of n values (FP64/FP32) into out[0] (FP64); ``partial`` holds 1024 FP64.
hipError_t launch_sumsq(bool f32, const void* x, int64_t n, double* partial, double* out,
                        hipStream_t s);

// ---- als.hip --------------------------------------------------------------------------
struct Chain {
  int L;
  const double* core[8];
  int I[8];
  int Ra[8];
  int Rb[8];
};
// For every index l (row-major over the chain's modes) the product of the slices,
// written [l][r][c] (transpose = 0) or [l][c][r] (transpose = 1).
hipError_t launch_chain(const Chain& ch, int64_t count, int transpose, double* out,
                        const int* done, hipStream_t s);

struct AlsGeom {
  int N, n, Kn, RR, Ra, Rb;
  int64_t J;
  int cycK[8];          // dims of the cyclic order after mode n (N-1 entries)
  int64_t cycStride[8]; // strides of P for those modes
  int64_t strideN;      // stride of mode n in P
};
int64_t als_chunks(const AlsGeom& g);
bool als_supported(int Kn, int RR);
hipError_t launch_als_partial(const double* P, const AlsGeom& g, const double* Bm,
                              double* part, int64_t chunks, const int* done, hipStream_t s);
hipError_t launch_als_reduce(const double* part, int64_t chunks, int nout, double* sum,
                             const int* done, hipStream_t s);
hipError_t launch_als_solve(double* MG, const AlsGeom& g, double* Zn, unsigned* status,
                            const int* done, hipStream_t s);
hipError_t launch_als_resid(const double* P, const AlsGeom& g, const double* Bm,
                            const double* Zn, double* part, int64_t chunks, const int* done,
                            hipStream_t s);
hipError_t launch_als_err(const double* part, int64_t chunks, const double* pn2, int sweep,
                          double tol, double* trace, int* sweeps_run, int* done,
                          hipStream_t s);
hipError_t launch_als_begin(int* done, int* sweeps_run, hipStream_t s);

// ---- eval.hip -------------------------------------------------------------------------
hipError_t launch_backproject(const double* Z, const double* Q, int Ra, int K, int64_t In,
                              int Rb, double* G, hipStream_t s);
// out[0] += sum (x - tr(L[il] Rt[ir]))^2, out[1] = sum x^2 (two-stage, fixed order)
hipError_t launch_residual(bool f32, const void* X, int64_t IL, int64_t IR, int RR,
                           const double* L, const double* RtT, double* partial, double* out,
                           hipStream_t s);

}  // namespace rtr
