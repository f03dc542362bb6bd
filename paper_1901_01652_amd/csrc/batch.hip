// Batched TR-ALS (Alg. 1 step 9 for many small projected tensors at once): one persistent
// launch, one work-group per tensor, each work-group runs every sweep of its tensor's
// TR-ALS with the cores held in LDS.  Per core update n (Eq. 2 restricted to P):
//   M = P_<n> B      (K'_n x R_n R_{n+1}), B[j, (a,b)] = S_j[b, a] the subchain of the other
//                    cores; B is built tile by tile from a shared prefix Z_{n+1} .. Z_{n-2}
//                    times the last core of the chain, and M accumulated on the FP64 matrix
//                    cores;
//   G = B^T B        from the transfer matrices E_m = sum_i Z_m(i) (x) Z_m(i):
//                    sum_j S_j (x) S_j = E_{n+1} .. E_{n-1};
//   solve G W = M^T  Gauss-Jordan on the work-group, Z_n[a, i, b] = W[(a,b), i].
// The per-sweep error is explicit: ||P - Psi(Z)||^2 is accumulated tile by tile in the first
// tile pass of the next sweep (the subchain rows of core 1 with the current core 1 give
// Psi(Z) for those columns), and a final pass after the last sweep closes it.  The Gram
// identity ||P||^2 - 2 <M, W> + <W, G W> is not used: it cancels to ~1e-10 relative when the
// fit is good.
#include "common.hpp"
#include "launch.hpp"
#include "mfma.hpp"
#include "solve.hpp"

namespace rtr {

namespace {

constexpr int kBT = 256;  // threads per work-group (4 wavefronts)

__device__ __forceinline__ int64_t prefix_base(int q, const int* cyc, int ncyc,
                                               const int* K, const int64_t* stride) {
  // q is row-major over the cyclic modes cyc[0 .. ncyc-1] (cyc[0] slowest)
  int64_t off = 0;
  for (int t = ncyc - 1; t >= 0; --t) {
    const int m = cyc[t];
    const int km = K[m];
    const int x = q % km;
    q /= km;
    off += (int64_t)x * stride[m];
  }
  return off;
}

}  // namespace

// MQ: 16x16 output tiles of M per wavefront; GQ: Gauss-Jordan elements per thread.
template <int MQ, int GQ>
__global__ __launch_bounds__(kBT) void als_batch_kernel(const AlsItem* __restrict__ items,
                                                        int max_sweeps, double tol,
                                                        unsigned* __restrict__ status,
                                                        BatchLayout lay) {
  extern __shared__ double sm[];
  __shared__ double red[16];
  __shared__ int s_failed;
  const AlsItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = it.N;
  int K[8], R[8], zoff[9];
  int64_t stride[8];
  for (int n = 0; n < 8; ++n) {
    K[n] = n < N ? it.K[n] : 1;
    R[n] = n < N ? it.R[n] : 1;
  }
  zoff[0] = 0;
  for (int n = 0; n < N; ++n) zoff[n + 1] = zoff[n] + R[n] * K[n] * R[(n + 1) % N];
  stride[N - 1] = 1;
  for (int n = N - 2; n >= 0; --n) stride[n] = stride[n + 1] * K[n + 1];
  const int64_t total = stride[0] * K[0];

  double* Zs = sm;                     // cores, packed
  double* Ps = sm + lay.ps;            // P tile, [lay.kpad][lay.tj]
  double* Pre = sm + lay.pre;          // prefix rows [pq][b][c]
  double* Bs = sm + lay.bs;            // B tile, [lay.tj][lay.rrpad]
  // after the tile loop the tile region holds [T | E | T2 | M]; the Gram is then formed in
  // E's place and the solution in T's place
  double* Tb = sm + lay.ps;            // transfer-matrix chain
  double* Eb = Tb + lay.tsz;
  double* T2 = Eb + lay.tsz;
  double* Ms = T2 + lay.tsz;           // M, K'_n x RR
  double* Gs = Eb;                     // Gram, RR x RR
  double* Xs = Tb;                     // solution, RR x K'_n
  double* rowbuf = sm + lay.buf;       // 2 x 256
  double* colbuf = rowbuf + 512;       // 2 x 256

  for (int e = tid; e < zoff[N]; e += kBT) Zs[e] = it.Zinit[e];
  double pp = 0.0;
  for (int64_t e = tid; e < total; e += kBT) {
    const double v = it.P[e];
    pp += v * v;
  }
  const double pn2 = block_sum(pp, red);
  if (tid == 0) s_failed = 0;
  __syncthreads();

  double prev = 0.0;
  int sweeps = 0;
  bool done = false;
  for (int sw = 0; sw <= max_sweeps && !done; ++sw) {
    for (int n = 0; n < N; ++n) {
      // the first update of sweep sw > 0 also measures ||P - Psi(Z)|| of the cores left by
      // sweep sw - 1 (core 0 is still the old one while its M is accumulated); the extra
      // iteration sw == max_sweeps only measures
      const bool want_res = (n == 0 && sw > 0);
      const bool want_m = sw < max_sweeps;
      const int Ra = R[n], Rb = R[(n + 1) % N], RR = Ra * Rb, Kn = K[n];
      int cyc[8];
      for (int t = 1; t < N; ++t) cyc[t - 1] = (n + t) % N;
      const int last = cyc[N - 2];
      const int Kl = K[last], Rl = R[last];  // last core: R_l x K_l x R_n
      const int npre = N - 2;                // prefix modes cyc[0 .. N-3]
      const int64_t J = total / Kn;
      const int nq = (int)(J / Kl);
      const int npt = lay.tj / Kl;           // prefixes per tile (>= 1)
      const double* Zl = Zs + zoff[last];
      const int mt = (Kn + 15) >> 4, nt = (RR + 15) >> 4;
      f64x4 acc[MQ];
#pragma unroll
      for (int k = 0; k < MQ; ++k) acc[k] = f64x4{0.0, 0.0, 0.0, 0.0};
      double res = 0.0;  // per-lane share of ||P - Psi(Z)||^2

      for (int q0 = 0; q0 < nq; q0 += npt) {
        const int nqt = min(npt, nq - q0);
        const int tj = nqt * Kl;
        const int tjp = (tj + 3) & ~3;
        // P tile (zero beyond tj up to the next multiple of 4)
        for (int e = tid; e < Kn * tjp; e += kBT) {
          const int i = e / tjp, jj = e - i * tjp;
          double v = 0.0;
          if (jj < tj) {
            const int pq = jj / Kl, il = jj - pq * Kl;
            v = it.P[(int64_t)i * stride[n] + prefix_base(q0 + pq, cyc, npre, K, stride) +
                     (int64_t)il * stride[last]];
          }
          Ps[i * lay.tj + jj] = v;
        }
        // prefix rows: e_b^T Z_{cyc0}(i) .. Z_{cyc[npre-1]}(i), length R_l
        for (int e = tid; e < nqt * Rb; e += kBT) {
          const int pq = e / Rb, b = e - pq * Rb;
          double v[8], w[8];
          int width;
          if (npre == 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = (c == b) ? 1.0 : 0.0;
            width = Rb;
          } else {
            int q = q0 + pq;
            int idx[8];
            for (int t = npre - 1; t >= 0; --t) {
              const int km = K[cyc[t]];
              idx[t] = q % km;
              q /= km;
            }
            int m = cyc[0];
            int rm = R[m], rn = R[(m + 1) % N];
            const double* z = Zs + zoff[m] + ((int64_t)b * K[m] + idx[0]) * rn;
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = c < rn ? z[c] : 0.0;
            width = rn;
            for (int t = 1; t < npre; ++t) {
              m = cyc[t];
              rm = R[m];
              rn = R[(m + 1) % N];
              const double* zt = Zs + zoff[m] + (int64_t)idx[t] * rn;  // + p * K_m * rn
#pragma unroll
              for (int c = 0; c < 8; ++c) w[c] = 0.0;
#pragma unroll
              for (int p = 0; p < 8; ++p) {
                if (p < rm) {
                  const double vp = v[p];
                  const double* row = zt + (int64_t)p * K[m] * rn;
#pragma unroll
                  for (int c = 0; c < 8; ++c)
                    if (c < rn) w[c] += vp * row[c];
                }
              }
#pragma unroll
              for (int c = 0; c < 8; ++c) v[c] = w[c];
              width = rn;
            }
          }
          double* dst = Pre + (pq * Rb + b) * 8;
#pragma unroll
          for (int c = 0; c < 8; ++c) dst[c] = c < width ? v[c] : 0.0;
        }
        __syncthreads();
        // B tile: Bs[jj][(a,b)] = sum_c Pre[pq][b][c] Z_l[c, il, a]; zero in the padding
        for (int e = tid; e < tjp * Rb; e += kBT) {
          const int jj = e / Rb, b = e - jj * Rb;
          double* brow = Bs + jj * lay.rrpad;
          if (jj >= tj) {
            for (int a = 0; a < Ra; ++a) brow[a * Rb + b] = 0.0;
            continue;
          }
          const int pq = jj / Kl, il = jj - pq * Kl;
          const double* pr = Pre + (pq * Rb + b) * 8;
          double pv[8];
#pragma unroll
          for (int c = 0; c < 8; ++c) pv[c] = pr[c];
          for (int a = 0; a < Ra; ++a) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (c < Rl) s += pv[c] * Zl[((int64_t)c * Kl + il) * Ra + a];
            brow[a * Rb + b] = s;
          }
        }
        __syncthreads();
        // M += P_tile B_tile on the FP64 matrix cores (16 x 16 tiles, 4-deep steps)
        if (want_m) {
#pragma unroll
          for (int k = 0; k < MQ; ++k) {
            const int t = wave + 4 * k;
            if (t < mt * nt) {
              const int ti = (t / nt) * 16, tb = (t % nt) * 16;
              const int row = ti + (lane & 15), col = tb + (lane & 15), g = lane >> 4;
              const bool rok = row < Kn, cok = col < RR;
              for (int k0 = 0; k0 < tjp; k0 += 4) {
                const double av = rok ? Ps[row * lay.tj + k0 + g] : 0.0;
                const double bv = cok ? Bs[(k0 + g) * lay.rrpad + col] : 0.0;
                acc[k] = mma_f64(av, bv, acc[k]);
              }
            }
          }
        }
        // Psi tile = Z_n (K'_n x RR) B_tile^T, residual against the P tile
        if (want_res) {
          const double* zn = Zs + zoff[n];
          const int ntj = (tj + 15) >> 4;
          for (int t = wave; t < mt * ntj; t += 4) {
            const int ti = (t / ntj) * 16, tc = (t % ntj) * 16;
            const int row = ti + (lane & 15), col = tc + (lane & 15), g = lane >> 4;
            const bool rok = row < Kn, cok = col < tj;
            f64x4 ps = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < RR; k0 += 4) {
              const int ab = k0 + g;
              double av = 0.0, bv = 0.0;
              if (ab < RR) {
                const int a = ab / Rb, b = ab - a * Rb;
                if (rok) av = zn[((int64_t)a * Kn + row) * Rb + b];
                if (cok) bv = Bs[col * lay.rrpad + ab];
              }
              ps = mma_f64(av, bv, ps);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = ti + 4 * r + g;
              if (i < Kn && cok) {
                const double d = Ps[i * lay.tj + col] - ps[r];
                res += d * d;
              }
            }
          }
        }
        __syncthreads();
      }
      if (want_res) {
        const double r2 = block_sum(res, red);
        const double e = pn2 > 0.0 ? sqrt(r2 / pn2) : 0.0;
        if (tid == 0) it.err[sw - 1] = e;
        sweeps = sw;
        if ((tol > 0.0 && sw >= 2 && fabs(e - prev) < tol) || sw == max_sweeps) done = true;
        prev = e;
      }
      if (done) break;
      // M to LDS (accumulator: C[4 r + g][lane & 15])
#pragma unroll
      for (int k = 0; k < MQ; ++k) {
        const int t = wave + 4 * k;
        if (t < mt * nt) {
          const int ti = (t / nt) * 16, tb = (t % nt) * 16;
          const int col = tb + (lane & 15), g = lane >> 4;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ti + 4 * r + g;
            if (row < Kn && col < RR) Ms[row * RR + col] = acc[k][r];
          }
        }
      }
      // Gram from the transfer matrices: T = E_{cyc0} E_{cyc1} .. E_{last}
      for (int t = 0; t < N - 1; ++t) {
        const int m = cyc[t];
        const int rm = R[m], rn = R[(m + 1) % N], km = K[m];
        const int er = rm * rm, ec = rn * rn;
        double* dst = (t == 0) ? Tb : Eb;
        const double* z = Zs + zoff[m];
        for (int e = tid; e < er * ec; e += kBT) {
          const int row = e / ec, col = e - row * ec;
          const int p = row / rm, p2 = row - p * rm, q = col / rn, q2 = col - q * rn;
          double s = 0.0;
          for (int i = 0; i < km; ++i)
            s += z[((int64_t)p * km + i) * rn + q] * z[((int64_t)p2 * km + i) * rn + q2];
          dst[row * ec + col] = s;
        }
        __syncthreads();
        if (t > 0) {
          // T (Rb^2 x er) * E (er x ec) -> T2, then back into T
          const int tr = Rb * Rb;
          for (int e = tid; e < tr * ec; e += kBT) {
            const int row = e / ec, col = e - row * ec;
            double s = 0.0;
            for (int x = 0; x < er; ++x) s += Tb[row * er + x] * Eb[x * ec + col];
            T2[row * ec + col] = s;
          }
          __syncthreads();
          for (int e = tid; e < tr * ec; e += kBT) Tb[e] = T2[e];
          __syncthreads();
        }
      }
      // G[(a,b),(a',b')] = T[(b,b'),(a,a')]
      for (int e = tid; e < RR * RR; e += kBT) {
        const int r1 = e / RR, r2 = e - r1 * RR;
        const int a = r1 / Rb, b = r1 - a * Rb, a2 = r2 / Rb, b2 = r2 - a2 * Rb;
        Gs[e] = Tb[(b * Rb + b2) * (Ra * Ra) + a * Ra + a2];
      }
      __syncthreads();
      if (gauss_jordan<GQ>(Gs, Ms, Xs, rowbuf, colbuf, RR, Kn, &s_failed)) {
        __syncthreads();
        double* zn = Zs + zoff[n];
        for (int e = tid; e < RR * Kn; e += kBT) {
          const int r = e / Kn, i = e - r * Kn;
          const int a = r / Rb, b = r - a * Rb;
          zn[((int64_t)a * Kn + i) * Rb + b] = Xs[e];
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < zoff[N]; e += kBT) it.Z[e] = Zs[e];
  if (tid == 0) {
    *it.sweeps = sweeps;
    if (s_failed) atomicOr(status, (unsigned)RTR_STATUS_CHOLESKY_FAILED);
  }
}

template <int MQ, int GQ>
static hipError_t launch_batch_t(const AlsItem* items, int count, int max_sweeps, double tol,
                                 unsigned* status, const BatchLayout& lay, hipStream_t s) {
  const size_t lds = (size_t)lay.total * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)als_batch_kernel<MQ, GQ>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((als_batch_kernel<MQ, GQ>), dim3(count), dim3(kBT), lds, s, items,
                     max_sweeps, tol, status, lay);
  return hipGetLastError();
}

template <int MQ>
static hipError_t launch_batch_g(int gq, const AlsItem* items, int count, int max_sweeps,
                                 double tol, unsigned* status, const BatchLayout& lay,
                                 hipStream_t s) {
  switch (gq) {
    case 4: return launch_batch_t<MQ, 4>(items, count, max_sweeps, tol, status, lay, s);
    case 8: return launch_batch_t<MQ, 8>(items, count, max_sweeps, tol, status, lay, s);
    default: return launch_batch_t<MQ, 16>(items, count, max_sweeps, tol, status, lay, s);
  }
}

bool batch_layout(int maxK, int maxRR, int maxR, int64_t maxZ, int minKl, BatchLayout* lay,
                  int* mq, int* gq) {
  if (maxK > 64 || maxR > 6 || maxRR > 36 || minKl < 1) return false;
  BatchLayout l{};
  l.kpad = (maxK + 15) & ~15;
  l.tj = 64;
  l.rrpad = (maxRR + 15) & ~15;
  const int npt = l.tj / minKl;
  // transfer matrices are up to R^2 x R^2; the solution (RR x K'_n) reuses the first one
  l.tsz = std::max(maxR * maxR * maxR * maxR, maxRR * maxK);
  int64_t off = (maxZ + 31) & ~(int64_t)31;
  l.ps = (int)off;
  l.pre = l.ps + l.kpad * l.tj;
  l.bs = l.pre + npt * 6 * 8;
  const int64_t tile = std::max((int64_t)l.kpad * l.tj + npt * 6 * 8 + (int64_t)(l.tj + 4) * l.rrpad,
                                (int64_t)3 * l.tsz + (int64_t)maxK * maxRR);
  off += tile;
  l.buf = (int)off;
  off += 1024;
  l.total = (int)off;
  if (l.total * 8 > 150 * 1024) return false;
  const int tiles = ((maxK + 15) / 16) * ((maxRR + 15) / 16);
  *mq = (tiles + 3) / 4;
  const int ne = maxRR * (maxRR + maxK);
  if (ne > 16 * kBT) return false;
  *gq = ne <= 4 * kBT ? 4 : ne <= 8 * kBT ? 8 : 16;
  *lay = l;
  return true;
}

hipError_t launch_als_batch(const AlsItem* items, int count, int max_sweeps, double tol,
                            unsigned* status, const BatchLayout& lay, int mq, int gq,
                            hipStream_t s) {
  prof_begin("als_batch", s);
  hipError_t e;
  switch (mq) {
    case 1: e = launch_batch_g<1>(gq, items, count, max_sweeps, tol, status, lay, s); break;
    case 2: e = launch_batch_g<2>(gq, items, count, max_sweeps, tol, status, lay, s); break;
    default: e = launch_batch_g<3>(gq, items, count, max_sweeps, tol, status, lay, s); break;
  }
  prof_end(s);
  return e;
}

}  // namespace rtr
