// Alg. 1 step 9 with TR-SVD (the rTR-SVD variant of Sec. 3/4): sequential truncated SVDs
// of the projected tensor P, in the manner of TT-SVD (Oseledets 2011) with the first rank
// split over the two ends of the ring (Zhao et al. 2016, the TR-SVD the paper cites).
//
// Each step works on a row-major matrix C (m x n) that lives in device memory:
//   1. Gram of the shorter side, A = C C^T (m <= n) or C^T C (m > n), d = min(m, n);
//   2. one work-group diagonalises A by cyclic Jacobi with the round-robin parallel order
//      (d/2 disjoint rotations per round), sorts the eigenvalues, picks the smallest rank r
//      whose discarded energy sum_{i >= r} lambda_i stays within the step's budget, applies
//      the rank caps and splits the first rank as R_1 R_2;
//   3. U (m x r) becomes the core, diag(s) V^T (r x n) the next C, each singular pair
//      signed so that the largest-magnitude entry of its left vector is positive.
// The sizes (m, n, d, r) are decided on the device and kept in SvdState, so the whole
// sequence is enqueued without a host round trip; grids are sized from host-side bounds.
#include "common.hpp"
#include "launch.hpp"

namespace rtr {

namespace {

constexpr int kJacobiSweeps = 40;
constexpr int kEigThreads = 1024;

__device__ __forceinline__ void split_rank(int r, int* a, int* b) {
  int s = (int)sqrt((double)r);
  while ((s + 1) * (s + 1) <= r) ++s;
  while (s * s > r) --s;
  while (r % s) --s;
  *a = s;
  *b = r / s;
}

}  // namespace

__global__ void svd_init_kernel(SvdState* st, const double* pn2, double eps, int N, int m,
                                int n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->m = m;
  st->n = n;
  st->d = m < n ? m : n;
  st->rows = m <= n;
  st->r = 0;
  st->capped = 0;
  st->pn2 = *pn2;
  st->delta2 = eps * eps * (*pn2) / N;
  st->err2 = 0.0;
  for (int i = 0; i < 8; ++i) st->ranks[i] = 0;
}

// A = C C^T (rows) or C^T C, d x d, one 32 x 32 output tile per work-group (256 threads,
// 2 x 2 outputs each), contraction staged through LDS in chunks of 32.
__global__ __launch_bounds__(256) void svd_gram_kernel(const SvdState* __restrict__ st,
                                                       const double* __restrict__ C,
                                                       double* __restrict__ A) {
  __shared__ double Ta[32][33], Tb[32][33];
  const int d = st->d, m = st->m, n = st->n, rows = st->rows;
  const int L = rows ? n : m;
  const int p0 = blockIdx.y * 32, q0 = blockIdx.x * 32;
  if (p0 >= d || q0 >= d) return;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int c0 = 0; c0 < L; c0 += 32) {
    for (int e = tid; e < 1024; e += 256) {
      int o, c;
      if (rows) {
        o = e >> 5;
        c = e & 31;
      } else {
        o = e & 31;
        c = e >> 5;
      }
      const int cc = c0 + c;
      double va = 0.0, vb = 0.0;
      if (cc < L) {
        if (p0 + o < d) va = rows ? C[(int64_t)(p0 + o) * n + cc] : C[(int64_t)cc * n + p0 + o];
        if (q0 + o < d) vb = rows ? C[(int64_t)(q0 + o) * n + cc] : C[(int64_t)cc * n + q0 + o];
      }
      Ta[o][c] = va;
      Tb[o][c] = vb;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 32; ++c) {
      const double a0 = Ta[ty][c], a1 = Ta[ty + 16][c];
      const double b0 = Tb[tx][c], b1 = Tb[tx + 16][c];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int p = p0 + ty + 16 * a, q = q0 + tx + 16 * b;
      if (p < d && q < d) A[p * d + q] = acc[a][b];
    }
}

// Symmetric eigen-decomposition of the d x d Gram A (cyclic Jacobi, Golub & Van Loan
// Alg. 8.5.2 / 8.5.3 with the parallel round-robin ordering), then the truncation of this
// step.  The homes of A and V follow the step's actual Gram size d (known on the device only):
// both in LDS for d <= kSvdLdsDim, A in LDS and V in the global workspace for d <=
// kSvdLdsADim, both in the workspace above that.  The rotation and ordering arrays follow A
// and V in the same dynamic LDS block (svd_eig_lds bytes cover every case).
__device__ __host__ inline size_t svd_eig_book(int d) {
  const int np = (d + 1) / 2;
  return (size_t)np * (4 * sizeof(double) + 2 * sizeof(int) + 1) + (size_t)(2 * d + 1) * sizeof(double) +
         (size_t)d * sizeof(int);
}

static size_t svd_eig_lds(int dmax) {
  auto both = [](int d) { return (size_t)(d * (d | 1) + d * d) * sizeof(double) + svd_eig_book(d); };
  if (dmax <= kSvdLdsDim) return both(dmax);
  const size_t a = (size_t)kSvdLdsADim * (kSvdLdsADim | 1) * sizeof(double) + svd_eig_book(kSvdLdsADim);
  const size_t b = both(kSvdLdsDim);
  return std::max(std::max(a, b), svd_eig_book(std::min(dmax, kSvdMaxDim)));
}

__global__ __launch_bounds__(kEigThreads) void svd_eig_kernel(SvdState* __restrict__ st,
                                                              double* __restrict__ Ag,
                                                              double* __restrict__ Vg,
                                                              double* __restrict__ W,
                                                              double* __restrict__ sv,
                                                              SvdCaps caps, int step) {
  extern __shared__ double smem[];
  __shared__ int s_any, s_r;
  __shared__ double s_abs;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int d = st->d;
  const int mode = d <= kSvdLdsDim ? 1 : d <= kSvdLdsADim ? 2 : 0;
  const int dd = d * d;
  // A in LDS with an odd pitch (in doubles), so that the column updates of lanes on
  // consecutive rows fall on different banks; V kept transposed (Vt[p][i] = V[i][p]), so that
  // its column updates are contiguous rows
  const int lda = mode != 0 ? (d | 1) : d;
  double* A = mode != 0 ? smem : Ag;
  double* Vt = mode == 1 ? smem + d * lda : Vg;
  const int nph = (d + 1) / 2;
  double* pr_c = smem + (mode == 1 ? d * lda + dd : mode == 2 ? d * lda : 0);
  double* pr_s = pr_c + nph;
  double* pr_dp = pr_s + nph;
  double* pr_dq = pr_dp + nph;
  double* lam = pr_dq + nph;
  double* tail = lam + d;
  int* pr_p = (int*)(tail + d + 1);
  int* pr_q = pr_p + nph;
  int* perm = pr_q + nph;
  unsigned char* pr_rot = (unsigned char*)(perm + d);
  for (int e = tid; e < dd; e += nth) {
    if (mode != 0) A[(e / d) * lda + e % d] = Ag[e];
    const int i = e / d, j = e - i * d;
    Vt[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < d; ++i) tr += fabs(A[i * lda + i]);
    s_abs = 1e-22 * tr;  // off-diagonal entries below this are negligible
  }
  __syncthreads();
  const double abs_tol = s_abs;
  const int dp = d + (d & 1);
  const int npairs = dp / 2;
  for (int sweep = 0; sweep < kJacobiSweeps && d > 1; ++sweep) {
    if (tid == 0) s_any = 0;
    __syncthreads();
    for (int k = 0; k < dp - 1; ++k) {
      if (tid < npairs) {
        int a, b;
        if (tid == 0) {
          a = dp - 1;
          b = k;
        } else {
          a = (k + tid) % (dp - 1);
          b = (k - tid + dp - 1) % (dp - 1);
        }
        const int p = a < b ? a : b, q = a < b ? b : a;
        unsigned char rot = 0;
        double c = 1.0, s = 0.0, dpp = 0.0, dqq = 0.0;
        if (q < d) {
          const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
          if (fabs(apq) > fmax(1e-15 * sqrt(fabs(app * aqq)), abs_tol)) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            dpp = app - t * apq;
            dqq = aqq + t * apq;
            rot = 1;
            s_any = 1;
          }
        }
        pr_p[tid] = p;
        pr_q[tid] = q;
        pr_c[tid] = c;
        pr_s[tid] = s;
        pr_dp[tid] = dpp;
        pr_dq[tid] = dqq;
        pr_rot[tid] = rot;
      }
      __syncthreads();
      // A <- J^T A J in one pass: the pairs partition the indices, so the 2 x 2 block of pair
      // t's rows and pair u's columns becomes J_t^T M J_u from its own four entries (a pair
      // left alone has c = 1, s = 0; the spare index of an odd d has no row or column).  The
      // pivot blocks (t = u) are set exactly.  V <- V J on the rows of Vt in the same phase.
      const int nb = npairs * npairs;
      for (int e = tid; e < nb; e += nth) {
        const int t = e / npairs, u = e - t * npairs;
        const bool rt = pr_rot[t] != 0, ru = pr_rot[u] != 0;
        if (!rt && !ru) continue;
        const int p = pr_p[t], q = pr_q[t], pu = pr_p[u], qu = pr_q[u];
        if (t == u) {
          A[p * lda + p] = pr_dp[t];
          A[q * lda + q] = pr_dq[t];
          A[p * lda + q] = 0.0;
          A[q * lda + p] = 0.0;
          continue;
        }
        const bool hq = q < d, hqu = qu < d;
        const double x = A[p * lda + pu], y = hqu ? A[p * lda + qu] : 0.0;
        const double z = hq ? A[q * lda + pu] : 0.0, w = hq && hqu ? A[q * lda + qu] : 0.0;
        const double ct = pr_c[t], st_ = pr_s[t], cu = pr_c[u], su = pr_s[u];
        const double a1 = ct * x - st_ * z, b1 = ct * y - st_ * w;
        const double a2 = st_ * x + ct * z, b2 = st_ * y + ct * w;
        A[p * lda + pu] = cu * a1 - su * b1;
        if (hqu) A[p * lda + qu] = su * a1 + cu * b1;
        if (hq) A[q * lda + pu] = cu * a2 - su * b2;
        if (hq && hqu) A[q * lda + qu] = su * a2 + cu * b2;
      }
      for (int e = tid; e < npairs * d; e += nth) {
        const int t = e / d, i = e - t * d;
        if (!pr_rot[t]) continue;
        const int p = pr_p[t], q = pr_q[t];
        const double c = pr_c[t], s = pr_s[t];
        const double vip = Vt[p * d + i], viq = Vt[q * d + i];
        Vt[p * d + i] = c * vip - s * viq;
        Vt[q * d + i] = s * vip + c * viq;
      }
      __syncthreads();
    }
    const int any = s_any;
    __syncthreads();
    if (!any) break;
  }
  // eigenvalues in descending order (ties by index)
  for (int i = tid; i < d; i += nth) lam[i] = A[i * lda + i];
  __syncthreads();
  double lsorted = 0.0;
  int myrank = -1;
  if (tid < d) {
    const double li = lam[tid];
    int rk = 0;
    for (int j = 0; j < d; ++j) rk += (lam[j] > li) || (lam[j] == li && j < tid);
    myrank = rk;
    lsorted = li;
  }
  __syncthreads();
  if (myrank >= 0) {
    perm[myrank] = tid;
    lam[myrank] = lsorted;
  }
  __syncthreads();
  if (tid == 0) {
    tail[d] = 0.0;
    for (int i = d - 1; i >= 0; --i) tail[i] = tail[i + 1] + fmax(lam[i], 0.0);
    const double budget = st->delta2 * (step == 0 ? 2.0 : 1.0);
    int r = d;
    for (int rr = 1; rr <= d; ++rr)
      if (rr == d || tail[rr] <= budget) {
        r = rr;
        break;
      }
    int capped = 0;
    if (step == 0) {
      int a = 1, b = 1, rr = r;
      for (; rr >= 1; --rr) {
        split_rank(rr, &a, &b);
        if (a <= caps.c[0] && b <= caps.c[1 % caps.N]) break;
      }
      if (rr != r) capped = 1;
      r = rr;
      st->ranks[0] = a;
      st->ranks[1] = b;
    } else {
      const int cap = caps.c[step + 1];
      if (r > cap) {
        r = cap;
        capped = 1;
      }
      st->ranks[step + 1] = r;
    }
    st->err2 += tail[r];
    st->r = r;
    if (capped) st->capped = 1;
    s_r = r;
  }
  __syncthreads();
  const int r = s_r;
  for (int e = tid; e < d * r; e += nth) {
    const int i = e / r, c = e - i * r;
    W[e] = Vt[perm[c] * d + i];
  }
  for (int c = tid; c < r; c += nth) sv[c] = sqrt(fmax(lam[c], 0.0));
}

// Core k from U and the next matrix from diag(s) V^T (grid-stride over both outputs).
// Step 0 writes the first core as (R_1, K_1, R_2) and the next matrix permuted to
// (R_2, K_2 .. K_N, R_1) so the ring closes through R_1.
__global__ __launch_bounds__(256) void svd_project_kernel(const SvdState* __restrict__ st,
                                                          const double* __restrict__ C,
                                                          const double* __restrict__ W,
                                                          const double* __restrict__ sv,
                                                          double* __restrict__ Z,
                                                          double* __restrict__ Cn, int step) {
  const int m = st->m, n = st->n, rows = st->rows, r = st->r;
  const int R1 = st->ranks[0], R2 = st->ranks[1];
  const int64_t nu = (int64_t)m * r, total = nu + (int64_t)r * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nu) {
      const int p = (int)(e / r), c = (int)(e - (int64_t)p * r);
      double u;
      if (rows) {
        u = W[(int64_t)p * r + c];
      } else {
        double acc = 0.0;
        const double* cp = C + (int64_t)p * n;
        for (int j = 0; j < n; ++j) acc += cp[j] * W[(int64_t)j * r + c];
        const double s = sv[c];
        u = s > 1e-150 ? acc / s : 0.0;
      }
      if (step == 0) {
        const int a = c / R2, b = c - a * R2;
        Z[((int64_t)a * m + p) * R2 + b] = u;
      } else {
        Z[(int64_t)p * r + c] = u;
      }
    } else {
      const int64_t f = e - nu;
      const int c = (int)(f / n), j = (int)(f - (int64_t)c * n);
      double v;
      if (rows) {
        double acc = 0.0;
        for (int p = 0; p < m; ++p) acc += W[(int64_t)p * r + c] * C[(int64_t)p * n + j];
        v = acc;
      } else {
        v = sv[c] * W[(int64_t)j * r + c];
      }
      if (step == 0) {
        const int a = c / R2, b = c - a * R2;
        Cn[((int64_t)b * n + j) * R1 + a] = v;
      } else {
        Cn[(int64_t)c * n + j] = v;
      }
    }
  }
}

// Sign rule of every kept singular pair: negate column c of U and row c of the next matrix
// unless the entry of U's column with the largest magnitude (the first such on ties) is
// positive.  The split first rank makes the later steps depend on these signs.  One
// work-group per column; (|u|, index) is reduced with a total order, so the choice does
// not depend on the reduction order.
__global__ __launch_bounds__(256) void svd_sign_kernel(const SvdState* __restrict__ st,
                                                       double* __restrict__ Z,
                                                       double* __restrict__ Cn, int step) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int m = st->m, n = st->n, r = st->r;
  const int R1 = st->ranks[0], R2 = st->ranks[1];
  const int c = blockIdx.x;
  if (c >= r) return;
  const int tid = threadIdx.x;
  const int a = step == 0 ? c / R2 : 0, b = step == 0 ? c - a * R2 : 0;
  auto uidx = [&](int p) -> int64_t {
    return step == 0 ? ((int64_t)a * m + p) * R2 + b : (int64_t)p * r + c;
  };
  double best = -1.0;
  int bidx = m;
  for (int p = tid; p < m; p += blockDim.x) {
    const double v = fabs(Z[uidx(p)]);
    if (v > best) {  // p increases within a thread, so the first maximum is kept
      best = v;
      bidx = p;
    }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      const double v2 = bv[tid + w];
      const int i2 = bi[tid + w];
      if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
        bv[tid] = v2;
        bi[tid] = i2;
      }
    }
    __syncthreads();
  }
  const int pm = bi[0];
  if (pm >= m || !(Z[uidx(pm)] < 0.0)) return;
  for (int p = tid; p < m; p += blockDim.x) Z[uidx(p)] = -Z[uidx(p)];
  for (int j = tid; j < n; j += blockDim.x) {
    const int64_t o = step == 0 ? ((int64_t)b * n + j) * R1 + a : (int64_t)c * n + j;
    Cn[o] = -Cn[o];
  }
}

// Shape of the next matrix: step 0 leaves (R_2 K_2) x (K_3 .. K_N R_1), later steps
// (r K_{k+1}) x (rest / K_{k+1}).
__global__ void svd_next_kernel(SvdState* st, int step, int Knext) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int m, n;
  if (step == 0) {
    m = st->ranks[1] * Knext;
    n = (st->n / Knext) * st->ranks[0];
  } else {
    m = st->r * Knext;
    n = st->n / Knext;
  }
  st->m = m;
  st->n = n;
  st->d = m < n ? m : n;
  st->rows = m <= n;
}

// The remaining matrix (R_N K_N) x R_1 is the last core; ranks and the relative error out.
__global__ __launch_bounds__(256) void svd_last_kernel(const SvdState* __restrict__ st,
                                                       const double* __restrict__ C,
                                                       double* __restrict__ Zlast, int N,
                                                       int* __restrict__ ranks_out,
                                                       double* __restrict__ err_out,
                                                       unsigned* __restrict__ status) {
  const int64_t total = (int64_t)st->m * st->n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    Zlast[e] = C[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int i = 0; i < N; ++i) ranks_out[i] = st->ranks[i];
    *err_out = st->pn2 > 0.0 ? sqrt(st->err2 / st->pn2) : 0.0;
    if (st->capped) atomicOr(status, (unsigned)RTR_STATUS_RANK_CAPPED);
  }
}

hipError_t launch_svd_init(SvdState* st, const double* pn2, double eps, int N, int m, int n,
                           hipStream_t s) {
  hipLaunchKernelGGL(svd_init_kernel, dim3(1), dim3(64), 0, s, st, pn2, eps, N, m, n);
  return hipGetLastError();
}

hipError_t launch_svd_step(SvdState* st, const double* C, double* A, double* V, double* W,
                           double* sv, const SvdCaps& caps, int step, int dmax, double* Z,
                           double* Cn, int Knext, hipStream_t s) {
  prof_begin("svd_gram", s);
  const unsigned tiles = (unsigned)((dmax + 31) / 32);
  hipLaunchKernelGGL(svd_gram_kernel, dim3(tiles, tiles), dim3(256), 0, s, st, C, A);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_begin("svd_eig", s);
  const size_t lds = svd_eig_lds(dmax);
  e = hipFuncSetAttribute((const void*)svd_eig_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(svd_eig_kernel, dim3(1), dim3(kEigThreads), lds, s, st, A, V, W, sv, caps,
                     step);
  prof_end(s);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_begin("svd_project", s);
  hipLaunchKernelGGL(svd_project_kernel, dim3(512), dim3(256), 0, s, st, C, W, sv, Z, Cn, step);
  hipLaunchKernelGGL(svd_sign_kernel, dim3((unsigned)dmax), dim3(256), 0, s, st, Z, Cn, step);
  prof_end(s);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(svd_next_kernel, dim3(1), dim3(64), 0, s, st, step, Knext);
  return hipGetLastError();
}

hipError_t launch_svd_last(const SvdState* st, const double* C, double* Zlast, int N,
                           int* ranks_out, double* err_out, unsigned* status, hipStream_t s) {
  hipLaunchKernelGGL(svd_last_kernel, dim3(64), dim3(256), 0, s, st, C, Zlast, N, ranks_out,
                     err_out, status);
  return hipGetLastError();
}

}  // namespace rtr
