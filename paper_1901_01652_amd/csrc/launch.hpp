// Host-side launchers of the gfx950 kernels (one translation unit per kernel family; the
// C ABI in runtime.hip calls only these).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtr {

enum Arith { kF64 = 0, kF32 = 1, kBF16 = 2, kFP8 = 3 };

// Stream word of the Gaussian test matrix of mode n (tag 1 in bits 24..31).
__host__ __device__ inline uint32_t omega_stream(int n) {
  return (1u << 24) | ((uint32_t)(n & 0xFF) << 16);
}

// Stream word of the Gaussian factor of mode m in the Khatri-Rao test matrix of mode n (tag 3).
__host__ __device__ inline uint32_t kr_stream(int n, int m) {
  return (3u << 24) | ((uint32_t)(n & 0xFF) << 16) | ((uint32_t)(m & 0xFF) << 8);
}

// Khatri-Rao structured test matrix of one mode: row j of M (the row-major index of the other
// modes' indices, first other mode slowest) is the element-wise product over the other modes
// m of row i_m of their Gaussian factor F_m (I_m x ld, row-major).  f == nullptr: the plain
// Gaussian test matrix.
struct KrArgs {
  const void* f;            // factor storage: FP32 for the FP32/BF16 passes, FP64 for FP64
  int nm;                   // number of other modes (N - 1)
  int dim[7];               // their sizes, in increasing mode order
  int64_t off[7];           // element offset of each factor in f
  int ld;                   // factor row length (the mode's K)
};

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
                                 void* partial, int64_t chunks, hipStream_t s, const KrArgs* kr = nullptr);
// Elements [start, start+count) of a Gaussian stream (FP64 or FP32 Box-Muller).
hipError_t launch_normals(bool f32, uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                          int64_t start, int64_t count, void* out, hipStream_t s);
// Fiber-form power step Y' = X_(n) (X_(n)^T Q), Q row-major In x K (FP64).
bool power_supported(Arith ar, const ModeView& v, int K);
int64_t power_chunks(Arith ar, const ModeView& v, int K);
hipError_t launch_power_partial(Arith ar, const void* X, const ModeView& v, int K,
                                const double* Q, void* partial, int64_t chunks,
                                hipStream_t s);
// ---- fastpass.hip: matrix-core sketch (op 0) / power step (op 1) over FP32 X ----------
// A sketch (op 0) of a mode with I_n above fast_pass_block_rows() runs one launch per row
// block [row0, row0 + rows); partials are then [grid][rows][K].  rows = 0: all rows.  A
// projection wider than fast_pass_block_k() runs one launch per column block [k0, k0 + K) of
// Ktot columns (Ktot = 0: K); partials are then [grid][rows][K] for that block.
bool fast_pass_supported(Arith ar, const ModeView& v, int K, int op);
int64_t fast_pass_block_rows();
int fast_pass_block_k(Arith ar, const ModeView& v, int K, int op);
int64_t fast_pass_grid(Arith ar, const ModeView& v, int K, int op, const void* X,
                       int64_t row0 = 0, int64_t rows = 0);
hipError_t launch_fast_pass(Arith ar, int op, const void* X, const ModeView& v, int K,
                            uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                            const double* Q, void* partial, int64_t grid, hipStream_t s,
                            int64_t row0 = 0, int64_t rows = 0, int Ktot = 0, int k0 = 0,
                            const KrArgs* kr = nullptr);
// ---- slab.hip: BF16 sketch (op 0) / power step (op 1) of the last two modes in one pass ---
// X viewed as A contiguous slabs of Ip x Iq; partials [grid][Ip][Kp] and [grid][Iq][Kq] (FP32).
bool slab_pass_supported(int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq, const void* X,
                         int op);
int64_t slab_pass_grid(int64_t A);
hipError_t launch_slab_pass(int op, const void* X, int64_t A, int64_t Ip, int64_t Iq, int Kp,
                            int Kq, uint64_t seed, uint32_t swp, uint32_t swq, uint32_t tensor_id,
                            const double* Qp, const double* Qq, float* partp, float* partq,
                            int64_t grid, hipStream_t s);
// ---- sketch.hip, work lists: the sketches of many tensors in one launch (FP32 X; FP32 or BF16
// arithmetic), then every job's partials summed into its Ycol (column-major In x K) in a second
// launch.  Job j owns grid blocks [block_start[j], block_start[j+1]) (host-built prefix sums).
struct SketchJob {
  const void* X;
  int64_t A, In, B;
  int K;
  uint32_t stream, tensor_id;
  uint64_t seed;
  int64_t ntiles, per, chunks;
  int nrb;
  void* partial;   // [chunks][In][K] FP32
  double* Ycol;
};
int64_t sketch_job_chunks(const ModeView& v, int K, int target);
void sketch_job_fill(SketchJob& g, const void* X, const ModeView& v, int K, uint64_t seed,
                     uint32_t stream_word, uint32_t tensor_id, int64_t chunks, void* partial,
                     double* Ycol);
int64_t sketch_job_blocks(const SketchJob& g);
hipError_t launch_sketch_list(Arith ar, const SketchJob* jobs, const int64_t* block_start,
                              int njobs, int64_t blocks, int64_t max_out, hipStream_t s);
// QR of every job's Ycol (K <= 256) into Qout[j] (row-major In x K), work[j]: In x K scratch.
hipError_t launch_qr_list(const SketchJob* jobs, double* const* work, double* const* Qout,
                          int njobs, hipStream_t s);
// ---- compress.hip, work list: one mode product for many tensors per launch.  kc (4, 16 or
// 64): outputs per thread, the tile the batched autotuner picks.
struct TtmJob {
  const void* in;
  int64_t A, In, B;
  int K;
  const double* Q;
  double* out;
};
int64_t ttm_job_blocks(const TtmJob& g, int kc);
hipError_t launch_ttm_list(Arith ar, bool first, int kc, const TtmJob* jobs,
                           const int64_t* block_start, int njobs, int64_t blocks, hipStream_t s);
// ---- kr_sketch.hip: BF16 sketch of every mode in one read of X with Khatri-Rao test
// matrices (order >= 3; the last two modes form the slabs).  Keff: K'_n per mode (K'_n = I_n:
// mode not projected).  F holds the factors F^(n)_m (I_m x K'_n row-major) at foff[n][m];
// part[n]: [grid][I_n][K'_n] FP32 partial sketches; xpart: [grid] partial sums of ||X||^2.
bool kr_allmode_supported(int order, const int64_t* dims, const int* Keff, const void* X);
int64_t kr_allmode_grid(int order, const int64_t* dims);
hipError_t launch_kr_allmode(const void* X, int order, const int64_t* dims, const int* Keff,
                             const float* F, const int64_t (*foff)[8], float* const* part,
                             double* xpart, int64_t grid, hipStream_t s);
// Fixed-order sum of partials into column-major Ycol (K x In storage, Ycol[k*ldy+i]; ldy = 0
// means In).
hipError_t launch_reduce_partials(Arith ar, const void* partial, int64_t chunks, int64_t In,
                                  int K, double* Ycol, hipStream_t s, int64_t ldy = 0);

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
// Fused first stage (compress_fast.hip): T[a] = Q1^T X_a Q2 over the last two modes.
bool compress_slab_supported(Arith ar, int64_t A, int64_t I1, int64_t I2, int K1, int K2);
hipError_t launch_compress_slab(Arith ar, const void* X, int64_t A, int64_t I1, int64_t I2,
                                int K1, int K2, const double* Q1, const double* Q2, double* T,
                                hipStream_t s);
// BF16 path with FP32 refinement, one wavefront per slab (compress_wave.hip): same output.
bool compress_wave_supported(int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq, const void* X);
hipError_t launch_compress_wave(const void* X, int64_t A, int64_t Ip, int64_t Iq, int Kp, int Kq,
                                const double* Qp, const double* Qq, double* T, hipStream_t s);
// Sum of squares of n values (FP64/FP32) into out[0] (FP64); ``partial`` holds 1024 FP64.
// Fixed-order sum of count doubles into *out (one work-group).
hipError_t launch_sum(const double* x, int64_t count, double* out, hipStream_t s);
hipError_t launch_sumsq(bool f32, const void* x, int64_t n, double* partial, double* out,
                        hipStream_t s);

// ---- coo.hip --------------------------------------------------------------------------
// A tensor given by its nonzeros: idx is nnz x N (row-major), val FP64 or FP32.
struct CooArgs {
  const int64_t* idx;
  const void* val;
  int f32;
  int64_t nnz;
  int N;
  int64_t dims[8];
  int K[8];          // sketch: projection size per mode, 0 for a kept mode
  double* Y[8];      // sketch: column-major I_n x K_n accumulators (zeroed by the caller)
  uint64_t seed;
  uint32_t tid;
  unsigned* status;
};
// The compression as one product: P (F x B) = A B^T over the nonzeros.
struct CooGemm {
  const double* Q[8];  // Q_n, I_n x Kp[n] row-major
  int Kp[8];
  int split;           // modes 0..split-1 index the rows of P's F x B view
  int64_t F, B;
  int64_t slices, chunk;
  double* part;        // slices x F x B
};
hipError_t launch_coo_sketch(const CooArgs& a, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
int64_t coo_slices(int64_t nnz, int64_t F, int64_t B, int64_t max_part);
hipError_t launch_coo_compress(const CooArgs& a, CooGemm g, double* P, hipStream_t s);

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

// ---- als2.hip: two kernels per core update -------------------------------------------
struct AlsArgs2 {
  const double* P;
  const double* Z;       // packed cores
  int N, n, Kn, Ra, Rb, RR;
  int64_t J;
  int cycK[8];           // dims of P in the cyclic order after mode n
  int64_t cycStride[8];  // their strides in P
  int64_t strideN;
  int chI[8];            // the same modes seen as the subchain's cores
  int chRb[8];
  int64_t chOff[8];      // offsets of those cores in Z
  int64_t zoffN;         // offset of core n in Z
  int mode;              // bit 0: accumulate M; bit 1: residual with core n
  int gram_direct;       // 1: Gram = B^T B accumulated here; 0: formed in the solve
  int64_t ztotal;        // packed core count (staged in LDS when zlds)
  int zlds;
  int64_t tiles_per_wg;
  double* part;          // [grid][nout + 1], nout = Kn*RR (+ RR*RR if gram_direct)
  const int* done;
  // gram_extra: one more work-group forms the transfer-matrix Gram of core n into gram_out
  // (RR x RR) while the others accumulate M
  int gram_extra;
  double* gram_out;
  int tdim;
  int64_t zoffs[8];
  int Kc[8], Rc[8];
};
struct AlsSolveArgs {
  const double* gram_in;  // Gram formed by the accumulation launch (NULL: form it here)
  const double* part;
  double* red;            // the records summed (M, then the Gram when accumulated directly)
  int kwin;               // right-hand sides per window of the blocked solve (set at launch)
  int nparts, Kn, RR, Rb, Ra;
  int gram_direct;
  int N, n;
  const double* Z;        // packed cores (transfer-matrix Gram)
  int64_t zoff[8];
  int Kc[8], Rc[8];       // dims of the cores and ranks R_1..R_N
  int tdim;               // transfer-matrix buffers are tdim x tdim (pad16(max R^2))
  int64_t ztotal;         // packed core count
  double* Zn;
  unsigned* status;
  int* done;
  int report_sweep;  // >= 0: the partials also carry that sweep's residual
  int report_only;
  const double* pn2;
  double* trace;
  int* sweeps_run;
  double tol;
};
int als2_tdim(int rmax);
bool als2_supported(int Kn, int RR, int64_t J, int64_t ztotal, int gram_direct, int tdim,
                    int maxK);
int64_t als2_parts(int Kn, int RR, int64_t J, int64_t ztotal);
hipError_t launch_als_accum(AlsArgs2 g, int rmax, hipStream_t s);
hipError_t launch_als_solve2(AlsSolveArgs g, hipStream_t s);

// One cooperative launch for a whole TR-ALS decomposition (als2.hip, als_persist_kernel).
struct AlsPersistArgs {
  const double* P;        // K_1 x .. x K_N row-major
  double* Z;              // packed cores: the initial cores in, the result out
  const double* pn2;      // ||P||_F^2
  double* part;           // [G][rec] partial records
  double* red;            // [rec] summed record
  unsigned* bar;          // grid-barrier arrival counter (zeroed before the launch)
  unsigned* status;
  double* trace;
  int* sweeps_run;
  double tol;
  int max_sweeps;
  int N;
  int K[8], R[8];
  int64_t zoff[8];
  int64_t strideP[8];
  int64_t total;
  int64_t ztotal;
  unsigned spin_limit;    // bound of a barrier wait (in sleeps of ~128 cycles)
  // filled by als_persist_plan
  int TJ, G, maxNe, rmax, maxK;
  int64_t ubuf;           // doubles of the per-work-group tile buffers
  int64_t rec;            // record length: K_n R R' (M) + (R R')^2 (Gram) + 1 (residual)
};
bool als_persist_plan(AlsPersistArgs* g, size_t* lds);
hipError_t launch_als_persist(const AlsPersistArgs& g, size_t lds, hipStream_t s);

__device__ __forceinline__ int64_t cyc_base_of(int N, const int* cycK, const int64_t* cycStride,
                                               int64_t j) {
  int64_t base = 0;
  for (int t = N - 2; t >= 0; --t) {
    const int64_t d = cycK[t];
    base += (j % d) * cycStride[t];
    j /= d;
  }
  return base;
}

// ---- eval.hip -------------------------------------------------------------------------
hipError_t launch_backproject(const double* Z, const double* Q, int Ra, int K, int64_t In,
                              int Rb, double* G, hipStream_t s);
// out[0] = sum (x - tr(L[il] Rt[ir]))^2, out[1] = sum x^2 (two-stage, fixed order).
// ``partial`` holds 2 residual_blocks(...) doubles; for FP32 X, ``lr32`` holds
// (IL + IR) * ceil4(RR) floats (FP32 copies of L and R^T).
int64_t residual_blocks(bool f32, int64_t IL, int64_t IR, int RR);
hipError_t launch_residual(bool f32, const void* X, int64_t IL, int64_t IR, int RR,
                           const double* L, const double* RtT, double* partial, float* lr32,
                           double* out, hipStream_t s);

// ---- svd.hip --------------------------------------------------------------------------
constexpr int kSvdMaxDim = 512;  // largest Gram size min(m, n) of a TR-SVD step
constexpr int kSvdLdsDim = 96;   // Gram sizes up to this are diagonalised in LDS
constexpr int kSvdLdsADim = 136; // up to this the Gram sits in LDS, its eigenvectors in HBM
struct SvdState {                // device-resident shape and bookkeeping of the sequence
  int m, n, d, rows, r, capped;
  int ranks[8];
  double pn2, delta2, err2;
};
struct SvdCaps {
  int N;
  int c[8];
};
hipError_t launch_svd_init(SvdState* st, const double* pn2, double eps, int N, int m, int n,
                           hipStream_t s);
// One truncated-SVD step: C (device dims) -> core written at Z, next matrix at Cn.
hipError_t launch_svd_step(SvdState* st, const double* C, double* A, double* V, double* W,
                           double* sv, const SvdCaps& caps, int step, int dmax, double* Z,
                           double* Cn, int Knext, hipStream_t s);
hipError_t launch_svd_last(const SvdState* st, const double* C, double* Zlast, int N,
                           int* ranks_out, double* err_out, unsigned* status, hipStream_t s);

// ---- batch.hip ------------------------------------------------------------------------
struct AlsItem {  // one tensor of a batched TR-ALS (device array of these)
  const double* P;
  const double* Zinit;
  double* Z;
  double* err;
  int* sweeps;
  int N;
  int K[8];
  int R[8];
};
struct BatchLayout {  // dynamic-LDS offsets (doubles) shared by every work-group
  int kpad, tj, rrpad, tsz, ps, pre, bs, buf, total;
};
// Layout for the batch maxima (K'_n <= 64, R_n <= 6); false if unsupported.
bool batch_layout(int maxK, int maxRR, int maxR, int64_t maxZ, int minKl, BatchLayout* lay,
                  int* mq, int* gq);
hipError_t launch_als_batch(const AlsItem* items, int count, int max_sweeps, double tol,
                            unsigned* status, const BatchLayout& lay, int mq, int gq,
                            hipStream_t s);

// ---- mlp.hip --------------------------------------------------------------------------
struct GemmArgs {  // C = op(A) op(B): A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
  const float* A;
  const float* B;
  float* part;  // [slices][M][N]
  int64_t M, N, K;
  int64_t sam, sak, sbk, sbn;
  int64_t kslice;
};
struct TrLoss4 {
  int K[4];
  int R[4];
  int zpad;  // floats reserved for the cores in LDS
};
int gemm_slices(int64_t M, int64_t N, int64_t K, int64_t* kslice);
hipError_t launch_gemm(bool bf, GemmArgs g, int slices, hipStream_t s);
hipError_t launch_epilogue(const float* part, int slices, int64_t M, int64_t N,
                           const float* bias, const float* mask, int mode, float* out,
                           hipStream_t s);
hipError_t launch_colsum(const float* G, int64_t M, int64_t N, float* out, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* m, float* v, int64_t n, double lr,
                       double b1, double b2, double eps, int t, hipStream_t s);
hipError_t launch_to_f64(const float* x, int64_t n, int64_t per_row, const double* pn2, int order,
                         double* y, hipStream_t s);
hipError_t launch_normalize(const double* P, int64_t d, int rows, float* out, hipStream_t s);
size_t tr_loss4_lds(const TrLoss4& sh);
hipError_t launch_core_loss(const float* y, const float* t, int dout, float gscale, int batch,
                            float* loss, float* dy, hipStream_t s);
hipError_t launch_tr_loss4(const float* y, const float* tgt, int dout, const TrLoss4& sh,
                           float gscale, int batch, float* loss, float* dy, hipStream_t s);

// ---- probe.hip: HBM read-stream probe -------------------------------------------------
int probe_blocks();
hipError_t launch_read_probe(const void* x, int64_t bytes, double* part, double* out,
                             hipStream_t s);

}  // namespace rtr
