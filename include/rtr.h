/*
 * rtr.h - C ABI of the gfx950 randomized tensor-ring decomposition library (librtr.so).
 *
 * Method: Yuan, Li, Cao, Zhao, "Randomized Tensor Ring Decomposition and Its Application to
 * Large-scale Data Reconstruction" (arXiv:1901.01652), Algorithm 1 (rTRD).  Problem
 * statement (Eq. 4): given a dense order-N tensor X, projection sizes K_n and TR-ranks
 * R_1..R_N, find cores G_n (R_n x I_n x R_{n+1}, R_{N+1} = R_1) minimising
 * ||X - Psi([G_n])||_F, where Psi evaluates Eq. (1).
 *
 * The five entry points are the stages of Algorithm 1:
 *   rtr_sketch       steps 3-6 (+ power iterations named after Alg. 1): Gaussian sketch
 *                    Y_n = X_(n) M_n, economy QR -> Q_n
 *   rtr_compress     step 7 read cumulatively (Eq. 3): P = X x_1 Q_1^T ... x_N Q_N^T
 *   rtr_decompose    step 9: TR-ALS (or TR-SVD) on the small tensor P -> cores Z_n
 *   rtr_backproject  steps 10-12: G_n = Z_n x_2 Q_n
 *   rtr_residual     Sec. 4 error measure: ||X - Psi([G_n])||_F^2 and ||X||_F^2
 *
 * Conventions shared by every call
 * --------------------------------
 * - Tensors are dense, row-major (last index fastest), 1 <= N <= RTR_MAX_ORDER modes
 *   (N >= 2 for the decomposition), every dimension >= 1.
 * - Mode-n unfolding X_(n): row i_n, column = row-major index of the other indices in
 *   their natural order (i_1..i_{n-1}, i_{n+1}..i_N).  TR unfolding X_<n>: columns are
 *   row-major over the cyclic order (i_{n+1}, .., i_N, i_1, .., i_{n-1}).
 * - Packed per-mode buffers: Q holds Q_1..Q_N back to back, Q_n row-major I_n x K'_n with
 *   K'_n = min(K_n, I_n), at offset sum_{m<n} I_m K'_m.  Core buffers hold cores back to
 *   back, core n row-major (R_n, D_n, R_{n+1}) with D_n = K'_n (Z) or I_n (G), at offset
 *   sum_{m<n} R_m D_m R_{m+1}.  P is row-major K'_1 x .. x K'_N.
 * - K_n >= I_n means mode n is not projected (Q_n = identity, K'_n = I_n).
 * - Precision: Q, P, Z, G and every scalar output are FP64.  X is FP64 or FP32.  The
 *   ``compute`` argument picks the arithmetic of the passes over X: RTR_F64 (X FP64),
 *   RTR_F32 (X FP32, FP32 products and accumulation), RTR_BF16 (X FP32 rounded to bf16 on
 *   load, bf16 products on the matrix cores, FP32 accumulation; the compression adds the
 *   FP32 refinement terms X_hi Q_lo + X_lo Q_hi), RTR_FP8_E4M3 (the sketch products with X
 *   and M rounded to OCP e4m3, values clamped to +-448 first, on the fp8 matrix cores with
 *   FP32 accumulation; power steps and the compression then run as for RTR_BF16; meant for
 *   data within the e4m3 range, |x| <= 448, which the caller can reach by scaling X since
 *   Q_n does not depend on the scale).  QR, power-iteration orthonormalisation and the ALS
 *   normal-equation solves are always FP64.
 * - Random numbers: the Gaussian matrix of Alg. 1 step 4 is never stored.  Entry (j, k)
 *   of M_n is element e = j*K'_n + k of the Philox4x32-10 stream with key (seed mod 2^32,
 *   seed >> 32) and counter (e>>2 low word, e>>2 high word, 0x01000000 | n << 16,
 *   tensor_id), Box-Muller on word pairs (w0,w1) -> lanes 0,1 and (w2,w3) -> lanes 2,3,
 *   uniforms (w + 1/2) 2^-32.
 *
 * Memory and execution
 * --------------------
 * - Every array argument named "device" is caller-owned device memory; the library reads
 *   or writes it only inside the work it enqueues and never frees it.  Each such pointer is
 *   checked before anything is enqueued: it must be memory of the handle's device
 *   (hipMalloc'd or managed) whose allocation holds at least the bytes the call accesses
 *   from that address; host memory (plain, pinned or registered) and memory of another
 *   device are refused with RTR_ERR_INVALID_ARG.  Host arrays
 *   (dims, K, R, options) are read before the call returns.
 * - Calls enqueue work on ``stream`` (a hipStream_t; NULL = the legacy default stream) and
 *   return without waiting, except where a call says it synchronises.
 * - The handle owns a device workspace grown on demand (growing synchronises the device)
 *   and released by rtr_destroy.  A handle is not thread-safe, and its workspace is shared
 *   by all its calls: issue a handle's calls on one stream, or synchronise between streams.
 * - Errors: argument checks happen before anything is enqueued and return
 *   RTR_ERR_INVALID_ARG / RTR_ERR_UNSUPPORTED with a message in rtr_last_error(h).  HIP
 *   failures return RTR_ERR_DEVICE.  No C++ exception crosses the ABI and nothing aborts.
 *   Numerical trouble found on the device (a Gram matrix that is not positive definite in
 *   TR-ALS) sets bits of a device status word read by rtr_status_sync.
 * - Results are deterministic: same inputs, seed and device give bitwise identical outputs
 *   (fixed-order reductions, no floating-point atomics).
 */
#ifndef RTR_H
#define RTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTR_MAX_ORDER 8
#define RTR_MAX_RANK 32
/* Fixed scratch of rtr_sketch_noalloc, per GPU (32 MiB). */
#define RTR_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

typedef enum {
  RTR_OK = 0,
  RTR_ERR_INVALID_ARG = 1,  /* a size, pointer or option is out of range */
  RTR_ERR_UNSUPPORTED = 2,  /* valid request outside what the library implements */
  RTR_ERR_OOM = 3,          /* workspace allocation failed */
  RTR_ERR_DEVICE = 4,       /* a HIP runtime call failed */
  RTR_ERR_NUMERICAL = 5,    /* device status word reported a numerical failure */
  RTR_ERR_INTERNAL = 6
} rtr_status;

typedef enum { RTR_F64 = 0, RTR_F32 = 1, RTR_BF16 = 2, RTR_FP8_E4M3 = 3 } rtr_dtype;

typedef enum { RTR_METHOD_ALS = 0, RTR_METHOD_SVD = 1 } rtr_method;

/* Device status word bits (rtr_status_sync). */
#define RTR_STATUS_CHOLESKY_FAILED 0x1u /* an ALS Gram matrix was not positive definite;
                                           that core update was skipped */
#define RTR_STATUS_RANK_CAPPED 0x2u     /* TR-SVD: a rank was lowered to its cap, so the
                                           error bound eps may not hold */
#define RTR_STATUS_SYNC_TIMEOUT 0x4u    /* a device-wide barrier of the single-launch TR-ALS
                                           did not complete within its bound; the launch
                                           ended early and its outputs are not valid */
#define RTR_STATUS_INDEX_RANGE 0x8u     /* a coordinate-list entry lay outside the tensor and
                                           was skipped */

typedef struct rtr_context* rtr_handle;

/* Create a handle bound to HIP device ``device``.  *out is set to NULL on failure. */
rtr_status rtr_create(int device, rtr_handle* out);

/* Destroy a handle: synchronises the device, frees the workspace.  NULL is accepted. */
rtr_status rtr_destroy(rtr_handle h);

/* Message of the last failed call on ``h`` ("" if none).  Valid until the next call. */
const char* rtr_last_error(rtr_handle h);

/* Static name of a status code. */
const char* rtr_status_string(rtr_status s);

/*
 * Alg. 1 steps 3-6 for every mode, plus ``power_iters`` rounds of subspace iteration
 * (Halko, Martinsson, Tropp 2011, Alg. 4.4; named after Alg. 1 as an option).
 *   X          device, row-major I_1 x .. x I_N, dtype x_dtype (RTR_F64 or RTR_F32)
 *   dims       host, N entries I_n >= 1
 *   K          host, N entries K_n >= 1 (K_n >= I_n: identity, no sketch for that mode)
 *   seed, tensor_id   select the Gaussian stream (see above)
 *   compute    RTR_F64 (needs X FP64), RTR_F32 or RTR_BF16 (need X FP32)
 *   Q          device, FP64, packed Q_n (I_n x K'_n, orthonormal columns, R_ii >= 0)
 * Y_n is formed from the original X for every mode.  With power_iters = q the result is
 * qr((X_(n) X_(n)^T)^q X_(n) M_n); each round re-orthonormalises once in FP64.
 * Limits: projected modes take K_n <= 256 with RTR_F32 / RTR_BF16 and K_n <= 64 with RTR_F64
 * (RTR_ERR_UNSUPPORTED otherwise); with power_iters > 0 a mode longer than 256 needs
 * I_n K_n <= 8192.
 */
rtr_status rtr_sketch(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                      const int64_t* dims, const int32_t* K, int32_t power_iters,
                      uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                      void* stream);

/*
 * rtr_sketch with a structured test matrix (the remark after Alg. 1 names structured
 * projections as an option): M_n is the Khatri-Rao (column-wise Kronecker) product of one
 * Gaussian factor F_m (I_m x K_n) per other mode m, so row j of M_n, j the row-major index of
 * the other modes' indices (first other mode slowest), is prod_{m != n} F_m[i_m, :].  F_m is
 * elements [0, I_m K_n) of Gaussian stream (seed, 0x03000000 | n << 16 | m << 8, tensor_id),
 * row-major; only sum_{m != n} I_m K_n normals are drawn per mode instead of
 * prod_{m != n} I_m K_n.  Arguments, limits, errors and the power iterations as rtr_sketch; the
 * factors take workspace of sum_{m != n} I_m K_n FP32 (FP64 for RTR_F64) values.
 * With RTR_BF16, order >= 3, the last two modes projected, 16 <= I_{N-1}, I_N <= 256,
 * I_N % 4 == 0, every K'_n <= 32, at least 256 slabs (prod_{m < N-1} I_m) and X 16-byte aligned,
 * the sketches of ALL modes come from one read of X: a slab S of the last two modes contributes
 * to mode n (one of the first N-2) the column sums of F^(n)_{N-1} o (S F^(n)_N) scaled by the
 * slab's factor entries, and to the last two modes S F and S^T F likewise.  Otherwise one pass
 * per mode as rtr_sketch.
 *   x_norm2    device, 1 FP64 (may be NULL): ||X||_F^2, formed inside that single pass (an
 *              extra pass over X otherwise)
 */
rtr_status rtr_sketch_kr(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                         const int64_t* dims, const int32_t* K, int32_t power_iters,
                         uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                         double* x_norm2, void* stream);

/*
 * Alg. 1 steps 3-8 with step 7 read sequentially: for n = 1..N the sketch of mode n is taken
 * of P^(n-1) = X x_1 Q_1^T .. x_{n-1} Q_{n-1}^T (its Gaussian M_n has prod_{i<n} K'_i
 * prod_{i>n} I_i rows, stream as for rtr_sketch), Q_n = qr(P^(n-1)_(n) M_n) with R_ii >= 0, and
 * P^(n) = P^(n-1) x_n Q_n^T; P = P^(N).  The first projected mode reads X in ``compute``
 * arithmetic, later modes read the FP64 intermediate in FP64.  No power iterations.
 *   X, x_dtype, order, dims, K, seed, tensor_id, compute   as for rtr_sketch
 *   Q          device, FP64, packed Q_n (I_n x K'_n)
 *   P          device, FP64, row-major K'_1 x .. x K'_N
 *   p_norm2    device, 1 FP64 (may be NULL): ||P||_F^2
 * Limits: K'_n <= 256 for the first projected mode (FP32/BF16), <= 64 for the others and for
 * RTR_F64 (RTR_ERR_UNSUPPORTED otherwise).
 */
rtr_status rtr_sketch_sequential(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                                 const int64_t* dims, const int32_t* K, uint64_t seed,
                                 uint32_t tensor_id, rtr_dtype compute, double* Q, double* P,
                                 double* p_norm2, void* stream);

/*
 * rtr_sketch for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels and results
 * as rtr_sketch (bitwise identical for the same inputs); it calls no hipMalloc, hipFree or
 * other allocating routine, and kernel timing (rtr_profile_enable) does not apply to it.
 * Its scratch (the partial sketches and the QR work arrays) is one fixed device array of
 * RTR_NOALLOC_SCRATCH_BYTES per GPU, set up by the first rtr_create on that device and held
 * until the process ends.  A request that needs more scratch than that returns
 * RTR_ERR_UNSUPPORTED before anything is enqueued; RTR_ERR_DEVICE if the array could not be
 * located on this device.  Every call of this entry point on one GPU shares that array, and
 * the array keeps the contents of the last call: calls that overlap in time on one GPU (other
 * streams, handles or threads) race, so the caller serialises them.
 */
rtr_status rtr_sketch_noalloc(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                              const int64_t* dims, const int32_t* K, int32_t power_iters,
                              uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                              void* stream);

/*
 * Alg. 1 step 7 read cumulatively (Eq. 3): P = X x_1 Q_1^T x_2 .. x_N Q_N^T.
 *   X, x_dtype, order, dims, K, compute   as for rtr_sketch
 *   Q          device, FP64, packed Q_n from rtr_sketch
 *   P          device, FP64, row-major K'_1 x .. x K'_N
 *   p_norm2    device, 1 FP64 (may be NULL): ||P||_F^2
 * Limits: K'_n <= 256.
 */
rtr_status rtr_compress(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                        const int64_t* dims, const int32_t* K, const double* Q,
                        rtr_dtype compute, double* P, double* p_norm2, void* stream);

/*
 * Alg. 1 steps 3-6 for a sparse tensor given by its nonzeros (coordinate list); the paper
 * names sparse tensors as future work (Sec. 5).  X is the sum over entries z of
 * values[z] e_{indices[z, 0]} (x) .. (x) e_{indices[z, N-1]} (repeated coordinates add).
 * Y_n = X_(n) M_n with the same Gaussian M_n as rtr_sketch (so a sparse tensor and its dense
 * form give the same Q_n), formed from the nonzeros in FP64: each nonzero adds values[z]
 * times row j_n of M_n to row i_n of Y_n, j_n its column of X_(n), M_n's row drawn where it is
 * used.  The additions are FP64 atomics, so results are reproducible to rounding, not bitwise.
 * Then the FP64 QR with R_ii >= 0 as rtr_sketch; no power iterations.
 *   indices      device, int64, nnz x N row-major coordinates (0-based); an entry outside the
 *                tensor is skipped and sets RTR_STATUS_INDEX_RANGE
 *   values       device, nnz values, RTR_F64 or RTR_F32 (values_dtype)
 *   nnz          number of entries (0 allowed)
 *   order, dims, K, seed, tensor_id, Q   as for rtr_sketch
 *   x_norm2      device, 1 FP64 (may be NULL): sum of values^2 (||X||_F^2 when the
 *                coordinates are distinct)
 * Limits: K'_n <= 256 (RTR_ERR_UNSUPPORTED otherwise).
 */
rtr_status rtr_sketch_coo(rtr_handle h, const int64_t* indices, const void* values,
                          rtr_dtype values_dtype, int64_t nnz, int32_t order, const int64_t* dims,
                          const int32_t* K, uint64_t seed, uint32_t tensor_id, double* Q,
                          double* x_norm2, void* stream);

/*
 * Alg. 1 step 7 (Eq. 3) for a tensor given by its nonzeros, in FP64:
 * P = sum_z values[z] Q_1[i_1, :] (x) .. (x) Q_N[i_N, :].  Viewing P as an F x B matrix
 * (leading modes as rows), it is a product A B^T over the nonzeros, formed on the FP64 matrix
 * cores in slices of the nonzeros whose partial P are summed in a fixed order (bitwise
 * reproducible).
 *   indices, values, values_dtype, nnz, order, dims, K   as for rtr_sketch_coo
 *   Q          device, FP64, packed Q_n (I_n x K'_n)
 *   P          device, FP64, row-major K'_1 x .. x K'_N
 *   p_norm2    device, 1 FP64 (may be NULL): ||P||_F^2
 * Limits: order >= 2, prod K'_n <= 2^28 (RTR_ERR_UNSUPPORTED otherwise).
 */
rtr_status rtr_compress_coo(rtr_handle h, const int64_t* indices, const void* values,
                            rtr_dtype values_dtype, int64_t nnz, int32_t order, const int64_t* dims,
                            const int32_t* K, const double* Q, double* P, double* p_norm2,
                            void* stream);

typedef struct {
  rtr_method method;  /* RTR_METHOD_ALS or RTR_METHOD_SVD */
  int32_t max_sweeps; /* ALS: sweeps over n = 1..N (>= 1) */
  double tol;         /* ALS: stop after sweep s >= 2 once |e(s) - e(s-1)| < tol; 0 = off */
  double eps;         /* SVD: relative error bound ||P - Psi(Z)|| <= eps ||P|| */
} rtr_decompose_opts;

/*
 * Alg. 1 step 9 on the projected tensor P (row-major K'_1 x .. x K'_N, FP64, device).
 *   Kp         host, N entries K'_n (the dimensions of P)
 *   R          host, N ranks R_1..R_N (R_{N+1} = R_1), 1 <= R_n <= RTR_MAX_RANK and
 *              R_n R_{n+1} <= prod_{m != n} K'_m (each core's least squares is well posed)
 *   Z_init     device, packed initial cores (R_n, K'_n, R_{n+1}); random N(0,1) init or a
 *              warm start.  May alias Z.
 *   Z          device, packed output cores (same layout)
 *   err_trace  device, max_sweeps FP64: ||P - Psi(Z)||_F / ||P||_F after each sweep
 *              (entries after the last sweep run are left untouched)
 *   sweeps_run device, 1 int32: sweeps performed
 * TR-ALS updates core n by the exact least-squares solution of Eq. (2) restricted to P
 * (normal equations in FP64, solved by Gauss-Jordan elimination without pivoting on
 * [Gram | M^T]: every pivot of a positive-definite Gram is a positive Schur-complement
 * diagonal, so the solution is the Cholesky one; systems whose augmented rows exceed 256
 * entries use an FP64 Cholesky factorisation instead).  A Gram matrix that is not positive
 * definite (a non-positive pivot) sets RTR_STATUS_CHOLESKY_FAILED and leaves that core
 * unchanged.
 * Limits: K'_n <= 1024 and R_n R_{n+1} <= 256 (RTR_ERR_UNSUPPORTED otherwise).  With K'_n = I_n
 * (P = X in FP64) this is plain TR-ALS on the full tensor.
 * RTR_METHOD_SVD is rejected with RTR_ERR_INVALID_ARG: TR-SVD chooses the ranks, so it has
 * its own entry point, rtr_decompose_svd.
 */
rtr_status rtr_decompose(rtr_handle h, const double* P, int32_t order, const int32_t* Kp,
                         const int32_t* R, const rtr_decompose_opts* opts,
                         const double* Z_init, double* Z, double* err_trace,
                         int32_t* sweeps_run, void* stream);

/*
 * How rtr_decompose runs TR-ALS on this handle.  mode 0 (default): the whole decomposition in
 * one cooperative launch (every work-group keeps the cores in LDS, grid barriers between the
 * phases of a core update) when every rank is at most 6, K'_n <= 64 and the cores fit; other
 * shapes, and devices that cannot hold the launch's work-groups at once, use mode 1.
 * mode 1: two launches per core update (accumulation of P_<n> B over column tiles, then the
 * solve).  Both compute the same least-squares updates; their sums run in different orders.
 */
rtr_status rtr_set_als_launch(rtr_handle h, int32_t mode);

/*
 * How rtr_batch_run runs the sketches and compressions of a batch on this handle.  on = 1
 * (default): as work lists over the whole batch where the batch takes them (see
 * rtr_batch_autotune); on = 0: rtr_sketch and rtr_compress per tensor, on 8 branch streams in
 * the captured graph.  Both compute the same quantities; their sums run in different orders.
 */
rtr_status rtr_batch_set_work_lists(rtr_handle h, int32_t on);

/*
 * Alg. 1 step 9 with TR-SVD (the rTR-SVD variant of Sec. 4): sequential truncated SVDs of
 * P (TT-SVD style, Zhao et al. 2016) with the ranks chosen from the error bound.
 *   P, order, Kp  as for rtr_decompose (FP64 device, row-major K'_1 x .. x K'_N)
 *   Rcap       host, N rank caps, 1 <= Rcap_n <= 512; they size the slots of Z
 *   eps        > 0: target ||P - Psi(Z)||_F <= eps ||P||_F
 *   Z          device FP64: N slots of Rcap_n * K'_n * Rcap_{n+1} doubles, in mode order;
 *              core n is stored packed (R_n, K'_n, R_{n+1}) at the start of its slot
 *   ranks      device, N int32: the chosen R_1..R_N
 *   err        device, 1 FP64: ||P - Psi(Z)||_F / ||P||_F, from the discarded singular
 *              energy (the truncations are orthogonal projections, so this is exact up to
 *              rounding)
 * Budget: every truncation keeps the smallest rank whose discarded singular values have
 * 2-norm <= delta = eps ||P|| / sqrt(N), the first one sqrt(2) delta; the first rank r is
 * split as R_1 R_2 = r with R_1 <= R_2 and R_2 - R_1 minimal; the last core closes the ring
 * through R_1.  A rank above its cap is lowered to the cap (the first, to the largest r whose
 * split fits R_1 <= Rcap_1, R_2 <= Rcap_2) and sets RTR_STATUS_RANK_CAPPED.
 * Every step diagonalises the Gram matrix of its shorter side; the host bounds these sizes
 * from the caps and returns RTR_ERR_UNSUPPORTED if one may exceed 512.
 */
rtr_status rtr_decompose_svd(rtr_handle h, const double* P, int32_t order, const int32_t* Kp,
                             const int32_t* Rcap, double eps, double* Z, int32_t* ranks,
                             double* err, void* stream);

/*
 * Batched Alg. 1 step 9: TR-ALS on many small projected tensors in ONE persistent launch
 * (one work-group per tensor runs all of that tensor's sweeps with its cores in LDS).
 * The per-tensor arithmetic is that of rtr_decompose (RTR_METHOD_ALS): exact least-squares
 * core updates by the normal equations in FP64 (Gauss-Jordan); err_trace[s] =
 * ||P - Psi(Z)|| / ||P|| after sweep s, computed explicitly (the residual of every entry of P
 * is accumulated in the tile pass that follows the sweep), stopping rule as there.
 * A Gram that is not positive definite skips that update and sets RTR_STATUS_CHOLESKY_FAILED.
 *   items      host array of count entries; every pointer in it is a device pointer
 *   Limits: 2 <= order <= 8, K'_n <= 64, R_n <= 6, R_n R_{n+1} <= prod_{m != n} K'_m, and the
 *   largest tensor's cores and tiles must fit one work-group's LDS (else UNSUPPORTED).
 */
typedef struct {
  const double* P;        /* device, row-major K'_1 x .. x K'_N */
  const double* Z_init;   /* device, packed initial cores (R_n, K'_n, R_{n+1}); may alias Z */
  double* Z;              /* device, packed output cores */
  double* err_trace;      /* device, max_sweeps FP64 */
  int32_t* sweeps_run;    /* device, 1 int32 */
  int32_t order;
  int32_t Kp[RTR_MAX_ORDER];
  int32_t R[RTR_MAX_ORDER];
} rtr_als_item;

rtr_status rtr_decompose_batch(rtr_handle h, const rtr_als_item* items, int32_t count,
                               int32_t max_sweeps, double tol, void* stream);

/*
 * Alg. 1 steps 3-12 for a batch of tensors: the sketch and compression of every tensor
 * (as work lists over the whole batch where rtr_batch_autotune describes them, else
 * rtr_sketch and rtr_compress per tensor on 8 branch streams inside a captured graph), one batched
 * TR-ALS launch (rtr_decompose_batch), per-tensor back-projection
 * (rtr_backproject, skipped where G is NULL).  With use_graph != 0 the whole sequence is
 * captured into a HIP graph the first time a given item array is seen (that call runs
 * eagerly) and later calls with an identical item array and parameters replay the graph
 * with one launch.  The handle keeps one such graph; a workspace reallocation invalidates it.
 *   items      host array; all pointers are device pointers, dims/K/R/seed as for the
 *              single-tensor calls (K'_n = min(K_n, I_n) sizes P, Z, Z_init)
 */
typedef struct {
  const void* X;          /* device, row-major I_1 x .. x I_N (x_dtype) */
  int32_t order;
  int64_t dims[RTR_MAX_ORDER];
  int32_t K[RTR_MAX_ORDER];
  int32_t R[RTR_MAX_ORDER];
  uint64_t seed;
  uint32_t tensor_id;
  const double* Z_init;   /* device, packed initial cores */
  double* Q;              /* device, packed Q_n (output) */
  double* P;              /* device, K'_1 x .. x K'_N (output) */
  double* Z;              /* device, packed cores (output) */
  double* G;              /* device, packed back-projected cores (output) or NULL */
  double* err_trace;      /* device, max_sweeps FP64 */
  int32_t* sweeps_run;    /* device, 1 int32 */
} rtr_batch_item;

rtr_status rtr_batch_run(rtr_handle h, const rtr_batch_item* items, int32_t count,
                         rtr_dtype x_dtype, rtr_dtype compute, int32_t power_iters,
                         int32_t max_sweeps, double tol, int32_t use_graph, void* stream);

/*
 * Tile choice for the batched work lists of rtr_batch_run (FP32 X, no power iterations, every
 * K'_n <= 64): there the sketches of every (tensor, mode) run as one launch over a job list,
 * their sums as one, every QR as one, and each mode product of the compression (Eq. 3, mode 1
 * first) for every tensor as one launch per mode.  This call times the candidates on the given
 * batch (HIP events, the mean of three runs after one untimed run): 16, 64 or 256 column-tile
 * chunks per sketch job, then 4, 16 or 64 outputs per thread of the mode products, keeps the
 * fastest pair in the handle for later rtr_batch_run calls, and writes the table
 *   table[0] chunks per sketch job, table[1] outputs per thread,
 *   table[2..4] sketch microseconds for 16 / 64 / 256, table[5..7] mode-product microseconds
 *   for 4 / 16 / 64
 * (host, 8 int32).  The outputs Q and P of the items are overwritten while timing.
 * RTR_ERR_UNSUPPORTED when the batch does not take the work lists.
 */
rtr_status rtr_batch_autotune(rtr_handle h, const rtr_batch_item* items, int32_t count,
                              rtr_dtype x_dtype, rtr_dtype compute, int32_t* table,
                              void* stream);

/*
 * Learned warm start for TR-ALS (an initialisation of Alg. 1 step 9): a multilayer
 * perceptron maps the normalised projected tensor P~ = P / ||P|| (row-major, flattened) to
 * the packed initial cores (R_n, K'_n, R_{n+1}).  Hidden layers h_l = relu(h_{l-1} W_l + b_l),
 * output y = h_{L-1} W_L + b_L; W_l is sizes[l] x sizes[l+1] row-major FP32 (device),
 * b_l has sizes[l+1] entries.  compute RTR_BF16 rounds both operands of every product to
 * bf16 (FP32 accumulation), RTR_F32 multiplies in FP32.  All arrays are device arrays
 * except sizes, K, R and the pointer arrays W, b, acts, dW, db (host arrays of device
 * pointers).  Training loss: mean over the batch of ||P~ - Psi(Z)||^2.
 */
/* out[r, :] = P[r, :] / ||P[r, :]|| (FP64 in, FP32 out), rows x dim. */
rtr_status rtr_mlp_normalize(rtr_handle h, const double* P, int64_t dim, int32_t rows,
                             float* out, void* stream);
/* y (batch x sizes[layers]) from x (batch x sizes[0]); acts[l] (batch x sizes[l+1]) keeps the
 * post-ReLU output of hidden layer l for the backward pass. */
rtr_status rtr_mlp_forward(rtr_handle h, int32_t layers, const int32_t* sizes,
                           const float* const* W, const float* const* b, const float* x,
                           int32_t batch, float* const* acts, float* y, rtr_dtype compute,
                           void* stream);
/* Supervised core loss per sample: loss[s] = ||y[s] - target[s]||^2 over the per_row packed
 * core entries, dy[s] = grad_scale * 2 (y[s] - target[s]).  The targets are cores the method
 * itself produced (TR-ALS on the normalised projected tensor from one fixed initial set of
 * cores, so the targets share one gauge).  y, target, dy: device batch x per_row FP32; loss:
 * device batch FP32. */
rtr_status rtr_mlp_core_loss(rtr_handle h, const float* y, const float* target, int32_t batch,
                             int64_t per_row, float grad_scale, float* loss, float* dy,
                             void* stream);
/* Order-4 TR loss per sample: loss[s] = ||target[s] - Psi(cores in y[s])||^2 and
 * dy[s] = grad_scale * d loss[s] / d y[s] (K, R: 4 entries, R_n <= 8). */
rtr_status rtr_mlp_tr_loss(rtr_handle h, const float* y, const float* target, int32_t batch,
                           const int32_t* K, const int32_t* R, float grad_scale, float* loss,
                           float* dy, void* stream);
/* dW[l], db[l] (overwritten) from dy through the layers of rtr_mlp_forward. */
rtr_status rtr_mlp_backward(rtr_handle h, int32_t layers, const int32_t* sizes,
                            const float* const* W, const float* x, int32_t batch,
                            const float* const* acts, const float* dy, float* const* dW,
                            float* const* db, rtr_dtype compute, void* stream);
/* One Adam step (Kingma & Ba 2015) on n FP32 parameters; step = 1, 2, .. */
rtr_status rtr_mlp_adam(rtr_handle h, float* w, const float* g, float* m, float* v, int64_t n,
                        double lr, double beta1, double beta2, double eps, int32_t step,
                        void* stream);
/* FP64 initial cores for rtr_decompose from the predictions y (rows x per_row):
 * Z[r, :] = y[r, :] * ||P_r||^(1/order) with ||P_r||^2 = p_norm2[r] (device; NULL: no scaling),
 * so that Psi(Z) approximates P_r rather than P_r / ||P_r|| (Psi is multilinear). */
rtr_status rtr_mlp_to_cores(rtr_handle h, const float* y, int64_t per_row, int32_t rows,
                            const double* p_norm2, int32_t order, double* Z, void* stream);

/*
 * Alg. 1 steps 10-12, read as the product over the physical mode: G_n = Z_n x_2 Q_n,
 * G_n[a, i, b] = sum_k Q_n[i, k] Z_n[a, k, b].
 *   dims, K, R host;  Z, Q device FP64 packed;  G device FP64 packed (R_n, I_n, R_{n+1}).
 */
rtr_status rtr_backproject(rtr_handle h, int32_t order, const int64_t* dims,
                           const int32_t* K, const int32_t* R, const double* Z,
                           const double* Q, double* G, void* stream);

/*
 * Sec. 4 error measure, explicit: out[0] = ||X - Psi([G_n])||_F^2, out[1] = ||X||_F^2,
 * accumulated in FP64 (RSE = sqrt(out[0] / out[1])).
 *   X device (x_dtype RTR_F64 / RTR_F32);  G device FP64 packed (R_n, I_n, R_{n+1});
 *   out device, 2 FP64.
 */
rtr_status rtr_residual(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                        const int64_t* dims, const int32_t* R, const double* G,
                        double* out, void* stream);

/*
 * The Gaussian stream behind the test matrices of Alg. 1 step 4 (see "Random numbers"
 * above): out[t] = element start + t of stream (seed, stream_word, tensor_id), t < count.
 * dtype RTR_F64 gives the FP64 Box-Muller values used by the FP64 sketch, RTR_F32 the FP32
 * values used by the FP32 sketch (the BF16 sketch rounds those to bf16).  The Gaussian
 * matrix of mode n is stream_word 0x01000000 | n << 16.
 *   out  device, count values of the given dtype.
 */
rtr_status rtr_normals(rtr_handle h, uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                       int64_t start, int64_t count, rtr_dtype dtype, void* out, void* stream);

/* Wait for ``stream``, read and clear the device status word.  *bits gets the
 * RTR_STATUS_* bits; returns RTR_ERR_NUMERICAL if any bit was set. */
rtr_status rtr_status_sync(rtr_handle h, void* stream, uint32_t* bits);

/*
 * Kernel timing with HIP events on the launch stream (off by default).  rtr_profile_enable
 * level 1 brackets each launch of the kernels that stream the large tensor X (sketch,
 * power step, first compression pass, residual) with two events, level 2 every kernel,
 * level 0 turns timing off.  rtr_profile_read synchronises the device and returns the
 * summed duration (ms) and launch count of kernel ``name``; rtr_profile_reset drops all
 * records.
 */
rtr_status rtr_profile_enable(rtr_handle h, int32_t on);
/*
 * Measurement helper: stream ``bytes`` of device memory at ``x`` once with 16-byte loads
 * over a persistent grid and write their sum (as FP32 values, FP64 total) to out[0].  Its
 * launch time, recorded as kernel "read_probe", is the device's achievable HBM read rate:
 * the measured peak the passes over X are compared against beside the published 8 TB/s.
 *   x    device, 16-byte aligned;  bytes a positive multiple of 16;  out device, 1 FP64.
 */
rtr_status rtr_read_probe(rtr_handle h, const void* x, int64_t bytes, double* out,
                          void* stream);
rtr_status rtr_profile_reset(rtr_handle h);
rtr_status rtr_profile_read(rtr_handle h, const char* name, double* total_ms,
                            int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* RTR_H */
