// Dense FP64 solve of the TR-ALS normal equations on one work-group (shared by the
// single-tensor and batched ALS kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace rtr {

// Gauss-Jordan elimination on the augmented matrix [Gram | M^T] (RR x (RR + Kn)), without
// pivoting (the Gram is symmetric positive definite, every pivot is a Schur-complement
// diagonal).  Thread t owns elements e = t + nth*q, q < QMAX, in registers.  Step k: the
// owners of row k and column k publish them to LDS (double-buffered), one barrier, then every
// element is updated.  Leaves [I | Gram^-1 M^T] and hands every solution entry (r, i) of
// Gram^-1 M^T to store(r, i, value); returns false on a non-positive pivot.
template <int QMAX, typename Store>
__device__ bool gauss_jordan(const double* G, const double* M, Store store, double* rowbuf,
                             double* colbuf, int RR, int Kn, int* failed) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int W = RR + Kn, ne = RR * W;
  double a[QMAX];
  int rr[QMAX], cc[QMAX];  // row (-1: no element) and column of each owned element
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int e = tid + nth * q;
    const bool ok = e < ne;
    rr[q] = ok ? e / W : -1;
    cc[q] = ok ? e % W : 0;
    a[q] = 0.0;
    if (ok) a[q] = cc[q] < RR ? G[rr[q] * RR + cc[q]] : M[(cc[q] - RR) * RR + rr[q]];
  }
  for (int k = 0; k < RR; ++k) {
    double* rb = rowbuf + (k & 1) * 256;
    double* cb = colbuf + (k & 1) * 256;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (rr[q] == k) rb[cc[q]] = a[q];
      if (cc[q] == k && rr[q] >= 0) cb[rr[q]] = a[q];
    }
    __syncthreads();
    // every read of the step at once (indices of absent elements point at valid entries),
    // then one wait: the step costs one LDS round trip, not one per element
    const double piv = rb[k];
    double rv[QMAX], cv[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      rv[q] = rb[cc[q]];
      cv[q] = cb[rr[q] > 0 ? rr[q] : 0];
    }
    if (!(piv > 0.0)) {
      if (tid == 0) *failed = 1;
      return false;
    }
    const double inv = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const double rk = rv[q] * inv;  // new row k entry
      const double up = (rr[q] == k) ? rk : fma(-cv[q], rk, a[q]);
      a[q] = rr[q] >= 0 ? up : a[q];
    }
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q)
    if (rr[q] >= 0 && cc[q] >= RR) store(rr[q], cc[q] - RR, a[q]);
  return true;
}

// The same with the solution written to X (RR x Kn, row-major).
template <int QMAX>
__device__ bool gauss_jordan(const double* G, const double* M, double* X, double* rowbuf,
                             double* colbuf, int RR, int Kn, int* failed) {
  return gauss_jordan<QMAX>(G, M, [=](int r, int i, double v) { X[r * Kn + i] = v; }, rowbuf,
                            colbuf, RR, Kn, failed);
}

}  // namespace rtr
