// Dense FP64 solve of the TR-ALS normal equations on one work-group (shared by the
// single-tensor and batched ALS kernels).
#pragma once
#include <hip/hip_runtime.h>

namespace rtr {

// Gauss-Jordan elimination on the augmented matrix [Gram | M^T] (RR x (RR + Kn)), without
// pivoting (the Gram is symmetric positive definite, every pivot is a Schur-complement
// diagonal).  Thread t owns elements e = t + nth*q, q < QMAX, in registers.  Step k: the
// owners of row k and column k publish them to LDS (double-buffered), one barrier, then every
// element is updated.  Leaves [I | Gram^-1 M^T]; returns false on a non-positive pivot.
template <int QMAX>
__device__ bool gauss_jordan(const double* G, const double* M, double* X, double* rowbuf,
                             double* colbuf, int RR, int Kn, int* failed) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int W = RR + Kn, ne = RR * W;
  double a[QMAX];
  int rr[QMAX], cc[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int e = tid + nth * q;
    rr[q] = e < ne ? e / W : -1;
    cc[q] = e % W;
    a[q] = 0.0;
    if (e < ne) a[q] = cc[q] < RR ? G[rr[q] * RR + cc[q]] : M[(cc[q] - RR) * RR + rr[q]];
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
    const double piv = rb[k];
    if (!(piv > 0.0)) {
      if (tid == 0) *failed = 1;
      return false;
    }
    const double inv = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      if (rr[q] >= 0) {
        const double rk = rb[cc[q]] * inv;  // new row k entry
        a[q] = (rr[q] == k) ? rk : a[q] - cb[rr[q]] * rk;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q)
    if (rr[q] >= 0 && cc[q] >= RR) X[rr[q] * Kn + (cc[q] - RR)] = a[q];
  return true;
}

}  // namespace rtr
