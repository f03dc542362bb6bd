// C ABI of librtr.so (include/rtr.h): argument checks, workspace, launch sequences of
// Algorithm 1's stages, kernel timing.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "launch.hpp"
#include "rtr.h"

// Scratch of the no-allocation sketch entry point (rtr_sketch_noalloc): one array per GPU the
// library runs on, held until the process ends.  In host code ``scratch`` names a host-side
// stand-in; its device address on each GPU comes from hipGetSymbolAddress (rtr_create) and is
// the only form host code passes on.
constexpr size_t kScratchBytes = RTR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of ``scratch`` per device ordinal
}  // namespace

struct ProfRec {
  const char* name;
  hipEvent_t e0, e1;
};

constexpr int kBatchBranches = 8;  // concurrent branches of a captured batch (16 measured no faster)

struct rtr_context {
  int device = 0;
  void* ws = nullptr;
  size_t ws_cap = 0;
  unsigned* status = nullptr;  // device status word
  std::string err;
  int prof_level = 0;  // 0 off, 1 kernels that stream the large tensor, 2 every kernel
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  const char* pending = nullptr;
  hipEvent_t pending_e0 = nullptr;
  int ws_epoch = 0;  // bumped whenever the workspace moves (cached graphs point into it)
  void* scratch = nullptr;  // device address of this device's no-allocation scratch
  int als_launch = 0;       // 0: single cooperative launch where supported, 1: per-update launches
  // batched TR-ALS: device item array, pinned staging for its upload
  void* items_dev = nullptr;
  size_t items_cap = 0;
  void* items_host = nullptr;
  size_t host_cap = 0;
  hipEvent_t items_copied = nullptr;
  // batched pipeline replayed as one graph
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t gkey = 0;
  int gepoch = -1;
  void* gitems_dev = nullptr;
  size_t gitems_cap = 0;
  // branch streams of the captured batch (default priority) and their fork/join events
  hipStream_t br[kBatchBranches] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kBatchBranches] = {};
  bool ws_locked = false;  // set while a capture hands out fixed slices of the workspace
  size_t ws_hi = 0;        // largest workspace request since it was last reset
  // batched work lists (sketch, QR, mode products of every tensor per launch): device job
  // arrays, and the tiles chosen by rtr_batch_autotune
  void* jobs_dev = nullptr;
  size_t jobs_cap = 0;
  int bt_target = 64;  // column-tile chunks per sketch job
  int bt_kc = 16;      // outputs per thread of the batched mode products
  int bt_lists = 1;    // rtr_batch_run may take the work lists
};

namespace {

thread_local rtr_context* g_ctx = nullptr;

struct Guard {  // makes the handle visible to the launchers' timing hooks
  explicit Guard(rtr_context* h) { g_ctx = h; }
  ~Guard() { g_ctx = nullptr; }
};

rtr_status fail(rtr_context* h, rtr_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

rtr_status hip_fail(rtr_context* h, hipError_t e, const char* what) {
  return fail(h, RTR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(h, e_, what); \
  } while (0)

hipEvent_t get_event(rtr_context* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Workspace: one device buffer, carved into 256-byte aligned regions per call.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

rtr_status ensure_ws(rtr_context* h, size_t bytes) {
  h->ws_hi = std::max(h->ws_hi, bytes);
  if (bytes <= h->ws_cap) return RTR_OK;
  if (h->ws_locked)
    return fail(h, RTR_ERR_INTERNAL, "workspace slice too small inside a graph capture");
  size_t cap = bytes + bytes / 8 + (1 << 20);
  if (h->ws) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_cap = 0;
  }
  ++h->ws_epoch;
  hipError_t e = hipMalloc(&h->ws, cap);
  if (e != hipSuccess) {
    h->ws = nullptr;
    (void)hipGetLastError();
    return fail(h, RTR_ERR_OOM, "workspace allocation of " + std::to_string(cap) + " bytes failed");
  }
  h->ws_cap = cap;
  return RTR_OK;
}

rtr_status check_handle(rtr_context* h) {
  if (!h) return RTR_ERR_INVALID_ARG;
  h->err.clear();
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
  return RTR_OK;
}

// A device array argument: memory of the handle's device (hipMalloc'd or managed) whose
// allocation covers [p, p + bytes).  Host memory (pinned, registered or plain) and memory of
// another device are rejected here, before anything is enqueued, instead of faulting a kernel.
// Where the runtime cannot report the allocation's extent the size check is skipped.
rtr_status check_dev(rtr_context* h, const void* p, size_t bytes, const char* what) {
  if (!p) return fail(h, RTR_ERR_INVALID_ARG, std::string(what) + " is NULL");
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, RTR_ERR_INVALID_ARG, std::string(what) + " is not device memory");
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(h, RTR_ERR_INVALID_ARG, std::string(what) + " is not device memory (memory type " +
                                            std::to_string((int)a.type) + ")");
  if (a.device != h->device)
    return fail(h, RTR_ERR_INVALID_ARG, std::string(what) + " is memory of device " +
                                            std::to_string(a.device) + ", not of the handle's device " +
                                            std::to_string(h->device));
  if (bytes > 0) {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return RTR_OK;
    }
    const uintptr_t end = (uintptr_t)base + size, q = (uintptr_t)p;
    if (q < (uintptr_t)base || bytes > end - q)
      return fail(h, RTR_ERR_INVALID_ARG, std::string(what) + " holds " + std::to_string(end - q) +
                                              " bytes from the given address, the call accesses " +
                                              std::to_string(bytes));
  }
  return RTR_OK;
}

// Optional device argument: NULL is accepted.
rtr_status check_dev_opt(rtr_context* h, const void* p, size_t bytes, const char* what) {
  return p ? check_dev(h, p, bytes, what) : RTR_OK;
}

#define CHECK_DEV(p, bytes, what)                             \
  do {                                                        \
    rtr_status s_ = check_dev(h, (p), (bytes), (what));       \
    if (s_) return s_;                                        \
  } while (0)

size_t x_bytes(const int64_t* dims, int order, rtr_dtype dt) {
  size_t z = dt == RTR_F64 ? 8 : 4;
  for (int n = 0; n < order; ++n) z *= (size_t)dims[n];
  return z;
}

rtr_status check_shape(rtr_context* h, int32_t order, const int64_t* dims, const int32_t* K) {
  if (order < 1 || order > RTR_MAX_ORDER)
    return fail(h, RTR_ERR_INVALID_ARG, "order must be in [1, " + std::to_string(RTR_MAX_ORDER) + "]");
  if (!dims) return fail(h, RTR_ERR_INVALID_ARG, "dims is NULL");
  for (int n = 0; n < order; ++n)
    if (dims[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, "dims[" + std::to_string(n) + "] < 1");
  if (K) {
    for (int n = 0; n < order; ++n)
      if (K[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, "K[" + std::to_string(n) + "] < 1");
  }
  return RTR_OK;
}

rtr_status check_arith(rtr_context* h, rtr_dtype x_dtype, rtr_dtype compute, rtr::Arith* ar) {
  if (x_dtype == RTR_F64 && compute == RTR_F64) {
    *ar = rtr::kF64;
    return RTR_OK;
  }
  if (x_dtype == RTR_F32 && compute == RTR_F32) {
    *ar = rtr::kF32;
    return RTR_OK;
  }
  if (x_dtype == RTR_F32 && compute == RTR_BF16) {
    *ar = rtr::kBF16;
    return RTR_OK;
  }
  if (x_dtype == RTR_F32 && compute == RTR_FP8_E4M3) {
    *ar = rtr::kFP8;
    return RTR_OK;
  }
  return fail(h, RTR_ERR_UNSUPPORTED,
              "supported (x_dtype, compute): (F64, F64), (F32, F32), (F32, BF16), (F32, FP8_E4M3)");
}

// The FP8 compute option applies to the sketch products only; power steps and mode products
// run in the bf16 arithmetic (with its FP32 refinement in the compression).
rtr::Arith not_fp8(rtr::Arith ar) { return ar == rtr::kFP8 ? rtr::kBF16 : ar; }

int64_t keff(const int64_t* dims, const int32_t* K, int n) {
  return K[n] < dims[n] ? (int64_t)K[n] : dims[n];
}

size_t q_bytes(const int64_t* dims, const int32_t* K, int order) {
  size_t z = 0;
  for (int n = 0; n < order; ++n) z += (size_t)dims[n] * keff(dims, K, n);
  return z * sizeof(double);
}

rtr::ModeView mode_view(const int64_t* dims, int order, int n) {
  rtr::ModeView v{1, dims[n], 1};
  for (int m = 0; m < n; ++m) v.A *= dims[m];
  for (int m = n + 1; m < order; ++m) v.B *= dims[m];
  return v;
}

}  // namespace

namespace rtr {
static bool streams_x(const char* name) {
  static const char* const kNames[] = {"sketch_partial", "power_partial", "ttm_first",
                                       "residual", "sketch_fused", "power_fused",
                                       "compress_fused", "read_probe", "als_persist",
                                       "sketch_slab", "power_slab", "sketch_kr_allmode"};
  for (const char* k : kNames)
    if (std::strcmp(k, name) == 0) return true;
  return false;
}

void prof_begin(const char* name, hipStream_t s) {
  rtr_context* h = g_ctx;
  if (!h || h->prof_level == 0) return;
  if (h->prof_level == 1 && !streams_x(name)) return;
  hipEvent_t e = get_event(h);
  if (!e) return;
  (void)hipEventRecord(e, s);
  h->pending = name;
  h->pending_e0 = e;
}
void prof_end(hipStream_t s) {
  rtr_context* h = g_ctx;
  if (!h || h->prof_level == 0 || !h->pending_e0) return;
  hipEvent_t e = get_event(h);
  if (!e) return;
  (void)hipEventRecord(e, s);
  h->recs.push_back(ProfRec{h->pending, h->pending_e0, e});
  h->pending = nullptr;
  h->pending_e0 = nullptr;
}
}  // namespace rtr

extern "C" {

rtr_status rtr_create(int device, rtr_handle* out) {
  if (!out) return RTR_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return RTR_ERR_INVALID_ARG;
  rtr_context* h = new (std::nothrow) rtr_context();
  if (!h) return RTR_ERR_OOM;
  h->device = device;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&h->status, sizeof(unsigned)) != hipSuccess ||
      hipMemset(h->status, 0, sizeof(unsigned)) != hipSuccess) {
    delete h;
    return RTR_ERR_DEVICE;
  }
  if (device < kMaxDevices) {  // once per device, with that device current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
        g_scratch_dev[device] = ptr;
      else
        (void)hipGetLastError();  // the no-allocation entry point then reports the failure
    }
    h->scratch = g_scratch_dev[device];
  }
  *out = h;
  return RTR_OK;
}

rtr_status rtr_destroy(rtr_handle h) {
  if (!h) return RTR_OK;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (int b = 0; b < kBatchBranches; ++b) {
    if (h->br[b]) (void)hipStreamDestroy(h->br[b]);
    if (h->join_ev[b]) (void)hipEventDestroy(h->join_ev[b]);
  }
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->items_copied) (void)hipEventDestroy(h->items_copied);
  if (h->items_dev) (void)hipFree(h->items_dev);
  if (h->gitems_dev) (void)hipFree(h->gitems_dev);
  if (h->jobs_dev) (void)hipFree(h->jobs_dev);
  if (h->items_host) (void)hipHostFree(h->items_host);
  if (h->ws) (void)hipFree(h->ws);
  if (h->status) (void)hipFree(h->status);
  delete h;
  return RTR_OK;
}

const char* rtr_last_error(rtr_handle h) { return h ? h->err.c_str() : "invalid handle"; }

const char* rtr_status_string(rtr_status s) {
  switch (s) {
    case RTR_OK: return "RTR_OK";
    case RTR_ERR_INVALID_ARG: return "RTR_ERR_INVALID_ARG";
    case RTR_ERR_UNSUPPORTED: return "RTR_ERR_UNSUPPORTED";
    case RTR_ERR_OOM: return "RTR_ERR_OOM";
    case RTR_ERR_DEVICE: return "RTR_ERR_DEVICE";
    case RTR_ERR_NUMERICAL: return "RTR_ERR_NUMERICAL";
    case RTR_ERR_INTERNAL: return "RTR_ERR_INTERNAL";
  }
  return "unknown";
}

// ---------------------------------------------------------------------------------------
namespace {

// Largest projection size: the QR kernel's limit (the sketch and the power step run in column
// blocks of at most 64).
constexpr int kSketchKMax = 256;

// Rows per block of the matrix-core sketch: equal blocks of at most fast_pass_block_rows(),
// rounded up to whole 16-row tiles.
int64_t row_block(int64_t In) {
  const int64_t cap = rtr::fast_pass_block_rows();
  if (In <= cap) return In;
  const int64_t nb = (In + cap - 1) / cap;
  return std::min(cap, ((In + nb - 1) / nb + 15) / 16 * 16);
}

// Alg. 1 steps 3-6 (+ power iterations).  With ``fixed`` the partial sketches and QR work
// arrays live in that buffer of ``fixed_cap`` bytes and nothing is allocated (a request that
// needs more is refused before anything is enqueued); otherwise in the handle's workspace.
rtr_status sketch_impl(rtr_context* h, const void* X, rtr_dtype x_dtype, int32_t order,
                       const int64_t* dims, const int32_t* K, int32_t power_iters, uint64_t seed,
                       uint32_t tensor_id, rtr_dtype compute, double* Q, void* stream,
                       void* fixed, size_t fixed_cap, bool khatri_rao = false,
                       double* x_norm2 = nullptr) {
  rtr_status st;
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K) return fail(h, RTR_ERR_INVALID_ARG, "K is NULL");
  if (power_iters < 0 || power_iters > 64)
    return fail(h, RTR_ERR_INVALID_ARG, "power_iters must be in [0, 64]");
  rtr::Arith ar;
  if ((st = check_arith(h, x_dtype, compute, &ar))) return st;
  CHECK_DEV(X, x_bytes(dims, order, x_dtype), "X");
  CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
  hipStream_t s = (hipStream_t)stream;

  // BF16 path: the last two modes share one slab pass per step (sketch, and each power round)
  // when both are projected and the slab shape fits the kernel
  const int sp = order - 2, sq = order - 1;
  int64_t slabA = 1;
  for (int n = 0; n < sp; ++n) slabA *= dims[n];
  const bool slab_ok = ar == rtr::kBF16 && !khatri_rao && order >= 2 &&
                       keff(dims, K, sp) < dims[sp] && keff(dims, K, sq) < dims[sq];
  const bool slab0 = slab_ok && rtr::slab_pass_supported(slabA, dims[sp], dims[sq], (int)keff(dims, K, sp),
                                                         (int)keff(dims, K, sq), X, 0);
  const bool slab1 = slab_ok && power_iters > 0 &&
                     rtr::slab_pass_supported(slabA, dims[sp], dims[sq], (int)keff(dims, K, sp),
                                              (int)keff(dims, K, sq), X, 1);
  const int64_t slab_grid = (slab0 || slab1) ? rtr::slab_pass_grid(slabA) : 0;
  const size_t slab_part = (size_t)slab_grid *
                           (size_t)(dims[sp] * keff(dims, K, sp) + dims[sq] * keff(dims, K, sq)) *
                           sizeof(float);
  // workspace: partial sums (largest mode), then per mode Ycol and Qwork
  const size_t pelem = (ar == rtr::kF64) ? sizeof(double) : sizeof(float);
  size_t pmax = (slab0 || slab1) ? slab_part : 0;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    if (k == dims[n]) continue;
    if (k > kSketchKMax)
      return fail(h, RTR_ERR_UNSUPPORTED,
                  "projection size above " + std::to_string(kSketchKMax) + " (mode " + std::to_string(n) + ")");
    rtr::ModeView v = mode_view(dims, order, n);
    size_t need = 0;
    const int kb = rtr::fast_pass_block_k(ar, v, (int)k, 0);
    if (kb > 0) {
      const int64_t rb = row_block(v.In);
      for (int64_t r0 = 0; r0 < v.In; r0 += rb) {
        const int64_t rows = std::min(rb, v.In - r0);
        need = std::max(need, (size_t)rtr::fast_pass_grid(ar, v, kb, 0, X, r0, rows) * rows * kb *
                                  sizeof(float));
      }
    } else {
      if (k > 64)
        return fail(h, RTR_ERR_UNSUPPORTED,
                    "projection size above 64 needs the FP32/BF16 path (mode " + std::to_string(n) + ")");
      need = (size_t)rtr::sketch_chunks(v, (int)k) * v.In * k * pelem;
    }
    if (power_iters > 0) {
      size_t pw;
      const rtr::Arith arp = not_fp8(ar);
      const int kb1 = rtr::fast_pass_block_k(arp, v, (int)k, 1);
      if (kb1 > 0) {
        pw = (size_t)rtr::fast_pass_grid(arp, v, kb1, 1, X) * v.In * kb1 * sizeof(float);
      } else {
        if (!rtr::power_supported(arp, v, (int)k))
          return fail(h, RTR_ERR_UNSUPPORTED,
                      "power iterations need I_n*K_n <= 8192 (mode " + std::to_string(n) + ")");
        pw = (size_t)rtr::power_chunks(arp, v, (int)k) * v.In * k * pelem;
      }
      if (pw > need) need = pw;
    }
    if (need > pmax) pmax = need;
  }
  // Khatri-Rao factors of one mode at a time (sum over the other modes of I_m K_n)
  size_t krmax = 0;
  if (khatri_rao)
    for (int n = 0; n < order; ++n) {
      size_t e = 0;
      for (int m = 0; m < order; ++m)
        if (m != n) e += (size_t)dims[m] * keff(dims, K, n);
      krmax = std::max(krmax, e * pelem);
    }
  // Khatri-Rao, BF16: every mode's sketch (and ||X||^2) in one pass when the slab shape fits
  int keffi[RTR_MAX_ORDER];
  for (int n = 0; n < order; ++n) keffi[n] = (int)keff(dims, K, n);
  const bool allmode = khatri_rao && ar == rtr::kBF16 && rtr::kr_allmode_supported(order, dims, keffi, X);
  const int64_t am_grid = allmode ? rtr::kr_allmode_grid(order, dims) : 0;
  size_t am_f = 0, am_p = 0;  // factor floats, partial floats
  int64_t am_foff[8][8] = {};
  if (allmode)
    for (int n = 0; n < order; ++n) {
      if (keffi[n] == dims[n]) continue;
      for (int m = 0; m < order; ++m) {
        if (m == n) continue;
        am_foff[n][m] = (int64_t)am_f;
        am_f += (size_t)dims[m] * keffi[n];
      }
      am_p += (size_t)am_grid * dims[n] * keffi[n];
    }
  Carve plan(nullptr);
  plan.take<char>(pmax);
  for (int n = 0; n < order; ++n) {
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
  }
  plan.take<char>(krmax);
  plan.take<float>(am_f);
  plan.take<float>(am_p);
  plan.take<double>((size_t)am_grid + 1024);
  void* ws;
  if (fixed) {
    if (plan.off + 256 > fixed_cap)
      return fail(h, RTR_ERR_UNSUPPORTED,
                  "this sketch needs " + std::to_string(plan.off + 256) + " bytes of scratch; the " +
                      "no-allocation entry point has " + std::to_string(fixed_cap));
    ws = fixed;
  } else {
    if ((st = ensure_ws(h, plan.off + 256))) return st;
    ws = h->ws;
  }
  Carve cv(ws);
  void* partial = cv.take<char>(pmax);
  // every launch below checks that its partial sums fit the planned buffer
  auto fits = [&](size_t bytes) -> rtr_status {
    return bytes <= pmax ? RTR_OK
                         : fail(h, RTR_ERR_INTERNAL, "partial sums exceed the planned workspace");
  };
  double* Ycol[RTR_MAX_ORDER];
  double* Qw[RTR_MAX_ORDER];
  double* Qn[RTR_MAX_ORDER];
  size_t qoff = 0;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    Ycol[n] = cv.take<double>((size_t)dims[n] * k);
    Qw[n] = cv.take<double>((size_t)dims[n] * k);
    Qn[n] = Q + qoff;
    qoff += (size_t)dims[n] * k;
  }
  void* krbuf = cv.take<char>(krmax);
  float* am_F = cv.take<float>(am_f);
  float* am_part = cv.take<float>(am_p);
  double* am_x = cv.take<double>((size_t)am_grid + 1024);
  // draws mode n's Khatri-Rao factors into krbuf and describes them
  auto kr_factors = [&](int n, rtr::KrArgs* ka) -> rtr_status {
    const int64_t k = keff(dims, K, n);
    *ka = rtr::KrArgs{};
    ka->f = krbuf;
    ka->ld = (int)k;
    int64_t off = 0;
    for (int m = 0; m < order; ++m) {
      if (m == n) continue;
      ka->dim[ka->nm] = (int)dims[m];
      ka->off[ka->nm] = off;
      ++ka->nm;
      char* dst = (char*)krbuf + off * pelem;
      HIP_TRY(rtr::launch_normals(pelem == sizeof(float), seed, rtr::kr_stream(n, m), tensor_id, 0,
                                  dims[m] * k, dst, s),
              "normals");
      off += dims[m] * k;
    }
    return RTR_OK;
  };

  rtr::QrJobs jobs{};
  // partial sums of the two slab modes (FP32) and the reduction of both into Ycol
  float* partp = (float*)partial;
  float* partq = partp + (size_t)slab_grid * dims[sp] * keff(dims, K, sp);
  auto reduce_slab = [&]() -> rtr_status {
    HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, partp, slab_grid, dims[sp], (int)keff(dims, K, sp),
                                        Ycol[sp], s), "reduce_partials");
    HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, partq, slab_grid, dims[sq], (int)keff(dims, K, sq),
                                        Ycol[sq], s), "reduce_partials");
    return RTR_OK;
  };
  if (allmode) {
    // every factor F^(n)_m, one pass over X, then each mode's partials into its Ycol
    float* parts[8] = {};
    size_t po = 0;
    for (int n = 0; n < order; ++n) {
      if (keffi[n] == dims[n]) continue;
      for (int m = 0; m < order; ++m)
        if (m != n)
          HIP_TRY(rtr::launch_normals(true, seed, rtr::kr_stream(n, m), tensor_id, 0,
                                      dims[m] * keffi[n], am_F + am_foff[n][m], s),
                  "normals");
      parts[n] = am_part + po;
      po += (size_t)am_grid * dims[n] * keffi[n];
    }
    HIP_TRY(rtr::launch_kr_allmode(X, order, dims, keffi, am_F, am_foff, parts, am_x, am_grid, s),
            "sketch_kr_allmode");
    if (x_norm2) HIP_TRY(rtr::launch_sum(am_x, am_grid, x_norm2, s), "sum");
  } else if (x_norm2) {
    size_t numel = 1;
    for (int n = 0; n < order; ++n) numel *= (size_t)dims[n];
    HIP_TRY(rtr::launch_sumsq(ar != rtr::kF64, X, (int64_t)numel, am_x, x_norm2, s), "sumsq");
  }
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    if (k == dims[n]) {
      HIP_TRY(rtr::launch_identity(Qn[n], dims[n], s), "identity");
      continue;
    }
    rtr::ModeView v = mode_view(dims, order, n);
    if (allmode) {
      size_t po = 0;
      for (int m = 0; m < n; ++m)
        if (keffi[m] < dims[m]) po += (size_t)am_grid * dims[m] * keffi[m];
      HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, am_part + po, am_grid, dims[n], (int)k, Ycol[n], s),
              "reduce_partials");
      const int j = jobs.count++;
      jobs.A[j] = Ycol[n];
      jobs.Qwork[j] = Qw[n];
      jobs.In[j] = dims[n];
      jobs.K[j] = (int)k;
      jobs.Q[j] = Qn[n];
      continue;
    }
    rtr::KrArgs ka{};
    if (khatri_rao && (st = kr_factors(n, &ka))) return st;
    const rtr::KrArgs* kp = khatri_rao ? &ka : nullptr;
    if (slab0 && (n == sp || n == sq)) {
      if (n == sp) {
        HIP_TRY(rtr::launch_slab_pass(0, X, slabA, dims[sp], dims[sq], (int)keff(dims, K, sp),
                                      (int)keff(dims, K, sq), seed, rtr::omega_stream(sp),
                                      rtr::omega_stream(sq), tensor_id, nullptr, nullptr, partp,
                                      partq, slab_grid, s),
                "sketch_slab");
        if ((st = reduce_slab())) return st;
      }
    } else if (rtr::fast_pass_supported(ar, v, (int)k, 0)) {
      // one launch per row block and column block (a single one when I_n and K_n fit)
      const int64_t rb = row_block(v.In);
      const int kmax = rtr::fast_pass_block_k(ar, v, (int)k, 0);
      for (int64_t r0 = 0; r0 < v.In; r0 += rb) {
        const int64_t rows = std::min(rb, v.In - r0);
        for (int k0 = 0; k0 < (int)k; k0 += kmax) {
          const int kb = std::min(kmax, (int)k - k0);
          const int64_t grid = rtr::fast_pass_grid(ar, v, kb, 0, X, r0, rows);
          if ((st = fits((size_t)grid * rows * kb * sizeof(float)))) return st;
          HIP_TRY(rtr::launch_fast_pass(ar, 0, X, v, kb, seed, rtr::omega_stream(n), tensor_id,
                                        nullptr, partial, grid, s, r0, rows, (int)k, k0, kp),
                  "sketch_fused");
          HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, partial, grid, rows, kb,
                                              Ycol[n] + (int64_t)k0 * v.In + r0, s, v.In),
                  "reduce_partials");
        }
      }
    } else {
      const int64_t chunks = rtr::sketch_chunks(v, (int)k);
      if ((st = fits((size_t)chunks * v.In * k * pelem))) return st;
      HIP_TRY(rtr::launch_sketch_partial(ar, X, v, (int)k, seed, rtr::omega_stream(n), tensor_id,
                                         partial, chunks, s, kp),
              "sketch_partial");
      HIP_TRY(rtr::launch_reduce_partials(ar, partial, chunks, v.In, (int)k, Ycol[n], s),
              "reduce_partials");
    }
    const int j = jobs.count++;
    jobs.A[j] = Ycol[n];
    jobs.Qwork[j] = Qw[n];
    jobs.In[j] = dims[n];
    jobs.K[j] = (int)k;
    jobs.Q[j] = Qn[n];
  }
  HIP_TRY(rtr::launch_householder_qr(jobs, s), "householder_qr");
  const rtr::Arith arp = not_fp8(ar);  // arithmetic of the power steps
  for (int it = 0; it < power_iters; ++it) {
    for (int n = 0; n < order; ++n) {
      const int64_t k = keff(dims, K, n);
      if (k == dims[n]) continue;
      rtr::ModeView v = mode_view(dims, order, n);
      if (slab1 && (n == sp || n == sq)) {
        if (n == sp) {
          HIP_TRY(rtr::launch_slab_pass(1, X, slabA, dims[sp], dims[sq], (int)keff(dims, K, sp),
                                        (int)keff(dims, K, sq), 0, 0, 0, 0, Qn[sp], Qn[sq], partp,
                                        partq, slab_grid, s),
                  "power_slab");
          if ((st = reduce_slab())) return st;
        }
      } else if (rtr::fast_pass_supported(arp, v, (int)k, 1)) {
        const int kmax = rtr::fast_pass_block_k(arp, v, (int)k, 1);
        for (int k0 = 0; k0 < (int)k; k0 += kmax) {
          const int kb = std::min(kmax, (int)k - k0);
          const int64_t grid = rtr::fast_pass_grid(arp, v, kb, 1, X);
          if ((st = fits((size_t)grid * v.In * kb * sizeof(float)))) return st;
          HIP_TRY(rtr::launch_fast_pass(arp, 1, X, v, kb, 0, 0, 0, Qn[n], partial, grid, s, 0, 0,
                                        (int)k, k0),
                  "power_fused");
          HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, partial, grid, v.In, kb,
                                              Ycol[n] + (int64_t)k0 * v.In, s, v.In),
                  "reduce_partials");
        }
      } else {
        const int64_t chunks = rtr::power_chunks(arp, v, (int)k);
        if ((st = fits((size_t)chunks * v.In * k * (arp == rtr::kF64 ? sizeof(double) : sizeof(float)))))
          return st;
        HIP_TRY(rtr::launch_power_partial(arp, X, v, (int)k, Qn[n], partial, chunks, s),
                "power_partial");
        HIP_TRY(rtr::launch_reduce_partials(arp, partial, chunks, v.In, (int)k, Ycol[n], s),
                "reduce_partials");
      }
    }
    HIP_TRY(rtr::launch_householder_qr(jobs, s), "householder_qr");
  }
  return RTR_OK;
}

}  // namespace

rtr_status rtr_sketch(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                      const int64_t* dims, const int32_t* K, int32_t power_iters,
                      uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                      void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  return sketch_impl(h, X, x_dtype, order, dims, K, power_iters, seed, tensor_id, compute, Q,
                     stream, nullptr, 0);
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_sketch_kr(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                         const int64_t* dims, const int32_t* K, int32_t power_iters,
                         uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                         double* x_norm2, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_dev_opt(h, x_norm2, sizeof(double), "x_norm2"))) return st;
  return sketch_impl(h, X, x_dtype, order, dims, K, power_iters, seed, tensor_id, compute, Q,
                     stream, nullptr, 0, true, x_norm2);
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_sketch_noalloc(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                              const int64_t* dims, const int32_t* K, int32_t power_iters,
                              uint64_t seed, uint32_t tensor_id, rtr_dtype compute, double* Q,
                              void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  // no Guard: the timing hooks stay off, so no event is created here
  if (!h->scratch)
    return fail(h, RTR_ERR_DEVICE, "the no-allocation scratch of this device is unavailable");
  return sketch_impl(h, X, x_dtype, order, dims, K, power_iters, seed, tensor_id, compute, Q,
                     stream, h->scratch, kScratchBytes);
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
namespace {
// Shared validation of a coordinate list: value type, count, device extents.
rtr_status check_coo(rtr_context* h, const int64_t* indices, const void* values,
                     rtr_dtype values_dtype, int64_t nnz, int32_t order) {
  if (values_dtype != RTR_F64 && values_dtype != RTR_F32)
    return fail(h, RTR_ERR_INVALID_ARG, "values_dtype must be RTR_F64 or RTR_F32");
  if (nnz < 0 || nnz > ((int64_t)1 << 40))
    return fail(h, RTR_ERR_INVALID_ARG, "nnz must be in [0, 2^40]");
  if (nnz > 0) {
    CHECK_DEV(indices, (size_t)nnz * order * sizeof(int64_t), "indices");
    CHECK_DEV(values, (size_t)nnz * (values_dtype == RTR_F64 ? 8 : 4), "values");
  }
  return RTR_OK;
}

rtr::CooArgs coo_args(rtr_context* h, const int64_t* indices, const void* values,
                      rtr_dtype values_dtype, int64_t nnz, int32_t order, const int64_t* dims) {
  rtr::CooArgs a{};
  a.idx = indices;
  a.val = values;
  a.f32 = values_dtype == RTR_F32 ? 1 : 0;
  a.nnz = nnz;
  a.N = order;
  for (int n = 0; n < order; ++n) a.dims[n] = dims[n];
  a.status = h->status;
  return a;
}
}  // namespace

rtr_status rtr_sketch_coo(rtr_handle h, const int64_t* indices, const void* values,
                          rtr_dtype values_dtype, int64_t nnz, int32_t order, const int64_t* dims,
                          const int32_t* K, uint64_t seed, uint32_t tensor_id, double* Q,
                          double* x_norm2, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K) return fail(h, RTR_ERR_INVALID_ARG, "K is NULL");
  if ((st = check_coo(h, indices, values, values_dtype, nnz, order))) return st;
  CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
  if ((st = check_dev_opt(h, x_norm2, sizeof(double), "x_norm2"))) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int n = 0; n < order; ++n)
    if (keff(dims, K, n) < dims[n] && keff(dims, K, n) > kSketchKMax)
      return fail(h, RTR_ERR_UNSUPPORTED,
                  "projection size above " + std::to_string(kSketchKMax) + " (mode " + std::to_string(n) + ")");
  Carve plan(nullptr);
  for (int n = 0; n < order; ++n) {
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
  }
  plan.take<double>(1024);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  rtr::CooArgs a = coo_args(h, indices, values, values_dtype, nnz, order, dims);
  a.seed = seed;
  a.tid = tensor_id;
  rtr::QrJobs jobs{};
  size_t qoff = 0;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    double* Y = cv.take<double>((size_t)dims[n] * k);
    double* Qw = cv.take<double>((size_t)dims[n] * k);
    double* Qn = Q + qoff;
    qoff += (size_t)dims[n] * k;
    if (k == dims[n]) {
      a.K[n] = 0;
      HIP_TRY(rtr::launch_identity(Qn, dims[n], s), "identity");
      continue;
    }
    a.K[n] = (int)k;
    a.Y[n] = Y;
    HIP_TRY(rtr::launch_fill(Y, dims[n] * k, 0.0, s), "fill");
    const int j = jobs.count++;
    jobs.A[j] = Y;
    jobs.Qwork[j] = Qw;
    jobs.In[j] = dims[n];
    jobs.K[j] = (int)k;
    jobs.Q[j] = Qn;
  }
  double* red = cv.take<double>(1024);
  HIP_TRY(rtr::launch_coo_sketch(a, s), "sketch_coo");
  HIP_TRY(rtr::launch_householder_qr(jobs, s), "householder_qr");
  if (x_norm2) {
    if (nnz > 0)
      HIP_TRY(rtr::launch_sumsq(values_dtype == RTR_F32, values, nnz, red, x_norm2, s), "sumsq");
    else
      HIP_TRY(rtr::launch_fill(x_norm2, 1, 0.0, s), "fill");
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_compress_coo(rtr_handle h, const int64_t* indices, const void* values,
                            rtr_dtype values_dtype, int64_t nnz, int32_t order, const int64_t* dims,
                            const int32_t* K, const double* Q, double* P, double* p_norm2,
                            void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K) return fail(h, RTR_ERR_INVALID_ARG, "K is NULL");
  if (order < 2) return fail(h, RTR_ERR_INVALID_ARG, "the coordinate-list compression needs order >= 2");
  if ((st = check_coo(h, indices, values, values_dtype, nnz, order))) return st;
  CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
  int64_t total = 1;
  for (int n = 0; n < order; ++n) total *= keff(dims, K, n);
  if (total > ((int64_t)1 << 28))
    return fail(h, RTR_ERR_UNSUPPORTED, "the projected tensor exceeds 2^28 entries");
  CHECK_DEV(P, (size_t)total * sizeof(double), "P");
  if ((st = check_dev_opt(h, p_norm2, sizeof(double), "p_norm2"))) return st;
  hipStream_t s = (hipStream_t)stream;
  // rows of P's F x B view: the leading modes that make F and B most even
  int split = 1;
  {
    int64_t best = -1, f = 1;
    for (int m = 1; m < order; ++m) {
      f *= keff(dims, K, m - 1);
      const int64_t b = total / f, worst = std::max(f, b);
      if (best < 0 || worst < best) {
        best = worst;
        split = m;
      }
    }
  }
  rtr::CooGemm g{};
  g.split = split;
  g.F = 1;
  size_t qoff = 0;
  for (int n = 0; n < order; ++n) {
    g.Q[n] = Q + qoff;
    g.Kp[n] = (int)keff(dims, K, n);
    qoff += (size_t)dims[n] * g.Kp[n];
    if (n < split) g.F *= g.Kp[n];
  }
  g.B = total / g.F;
  constexpr int64_t kPartMax = (int64_t)1 << 25;  // doubles of slice partials (256 MB)
  g.slices = rtr::coo_slices(nnz, g.F, g.B, std::max(kPartMax, total));
  Carve plan(nullptr);
  plan.take<double>((size_t)g.slices * total);
  plan.take<double>(1024);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  g.part = cv.take<double>((size_t)g.slices * total);
  double* red = cv.take<double>(1024);
  rtr::CooArgs a = coo_args(h, indices, values, values_dtype, nnz, order, dims);
  HIP_TRY(rtr::launch_coo_compress(a, g, P, s), "compress_coo");
  if (p_norm2) HIP_TRY(rtr::launch_sumsq(false, P, total, red, p_norm2, s), "sumsq");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_compress(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                        const int64_t* dims, const int32_t* K, const double* Q,
                        rtr_dtype compute, double* P, double* p_norm2, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K) return fail(h, RTR_ERR_INVALID_ARG, "K is NULL");
  rtr::Arith ar;
  if ((st = check_arith(h, x_dtype, compute, &ar))) return st;
  ar = not_fp8(ar);  // the compression reads X in bf16 with the FP32 refinement
  CHECK_DEV(X, x_bytes(dims, order, x_dtype), "X");
  CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
  {
    size_t pb = sizeof(double);
    for (int n = 0; n < order; ++n) pb *= (size_t)keff(dims, K, n);
    CHECK_DEV(P, pb, "P");
  }
  if ((st = check_dev_opt(h, p_norm2, sizeof(double), "p_norm2"))) return st;
  hipStream_t s = (hipStream_t)stream;
  for (int n = 0; n < order; ++n)
    if (keff(dims, K, n) > kSketchKMax)
      return fail(h, RTR_ERR_UNSUPPORTED,
                  "projection size above " + std::to_string(kSketchKMax) + " (mode " + std::to_string(n) + ")");
  size_t qoffs[RTR_MAX_ORDER];
  {
    size_t q = 0;
    for (int n = 0; n < order; ++n) {
      qoffs[n] = q;
      q += (size_t)dims[n] * keff(dims, K, n);
    }
  }
  // Plan: optionally the fused product over the last two modes first, then one mode
  // product per remaining mode (mode 1 first).  Each step maps ``cur`` dims to new dims.
  int64_t A = 1;
  for (int n = 0; n < order - 2; ++n) A *= dims[n];
  // BF16: one wavefront per slab (compress_wave.hip); else the work-group slab kernel
  const bool wavek =
      order >= 2 && ar == rtr::kBF16 &&
      rtr::compress_wave_supported(A, dims[order - 2], dims[order - 1], (int)keff(dims, K, order - 2),
                                   (int)keff(dims, K, order - 1), X);
  const bool fused =
      order >= 2 && (wavek || rtr::compress_slab_supported(ar, A, dims[order - 2], dims[order - 1],
                                                           (int)keff(dims, K, order - 2),
                                                           (int)keff(dims, K, order - 1)));
  int64_t cur[RTR_MAX_ORDER];
  for (int n = 0; n < order; ++n) cur[n] = dims[n];
  size_t maxmid = 1;
  auto numel = [&]() {
    size_t z = 1;
    for (int m = 0; m < order; ++m) z *= (size_t)cur[m];
    return z;
  };
  const int nmodes = fused ? order - 2 : order;  // modes left for single mode products
  if (fused) {
    cur[order - 2] = keff(dims, K, order - 2);
    cur[order - 1] = keff(dims, K, order - 1);
    if (nmodes > 0) maxmid = std::max(maxmid, numel());
  }
  for (int n = 0; n < nmodes - 1; ++n) {
    cur[n] = keff(dims, K, n);
    maxmid = std::max(maxmid, numel());
  }
  Carve plan(nullptr);
  plan.take<double>(maxmid);
  plan.take<double>(maxmid);
  plan.take<double>(1024);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  double* buf[2] = {cv.take<double>(maxmid), cv.take<double>(maxmid)};
  double* red = cv.take<double>(1024);

  for (int n = 0; n < order; ++n) cur[n] = dims[n];
  const void* in = X;
  bool in_is_x = true;
  int nb = 0;  // next ping-pong buffer
  if (fused) {
    const int K1 = (int)keff(dims, K, order - 2), K2 = (int)keff(dims, K, order - 1);
    double* out = (nmodes == 0) ? P : buf[nb];
    if (wavek)
      HIP_TRY(rtr::launch_compress_wave(X, A, dims[order - 2], dims[order - 1], K1, K2,
                                        Q + qoffs[order - 2], Q + qoffs[order - 1], out, s),
              "compress_fused");
    else
      HIP_TRY(rtr::launch_compress_slab(ar, X, A, dims[order - 2], dims[order - 1], K1, K2,
                                        Q + qoffs[order - 2], Q + qoffs[order - 1], out, s),
              "compress_fused");
    cur[order - 2] = K1;
    cur[order - 1] = K2;
    in = out;
    in_is_x = false;
    nb ^= 1;
  }
  for (int n = 0; n < nmodes; ++n) {
    const int64_t k = keff(dims, K, n);
    rtr::ModeView v = mode_view(cur, order, n);
    double* out = (n == nmodes - 1) ? P : buf[nb];
    HIP_TRY(rtr::launch_ttm(ar, in_is_x, in, v, (int)k, Q + qoffs[n], out, s), "ttm");
    cur[n] = k;
    in = out;
    in_is_x = false;
    nb ^= 1;
  }
  if (p_norm2) {
    size_t np = 1;
    for (int n = 0; n < order; ++n) np *= (size_t)cur[n];
    HIP_TRY(rtr::launch_sumsq(false, P, (int64_t)np, red, p_norm2, s), "sumsq");
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
// Alg. 1 steps 3-8 with step 7 read sequentially: mode n is sketched from the tensor already
// compressed in modes 1..n-1 (the first mode from X in the requested arithmetic, the later ones
// from the FP64 intermediate), then that tensor is multiplied by Q_n^T.
rtr_status rtr_sketch_sequential(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                                 const int64_t* dims, const int32_t* K, uint64_t seed,
                                 uint32_t tensor_id, rtr_dtype compute, double* Q, double* P,
                                 double* p_norm2, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K) return fail(h, RTR_ERR_INVALID_ARG, "K is NULL");
  rtr::Arith ar;
  if ((st = check_arith(h, x_dtype, compute, &ar))) return st;
  CHECK_DEV(X, x_bytes(dims, order, x_dtype), "X");
  CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
  size_t pnum = 1;
  for (int n = 0; n < order; ++n) pnum *= (size_t)keff(dims, K, n);
  CHECK_DEV(P, pnum * sizeof(double), "P");
  if ((st = check_dev_opt(h, p_norm2, sizeof(double), "p_norm2"))) return st;
  hipStream_t s = (hipStream_t)stream;

  // plan: dims of the tensor each projected mode sees, partial-sum sizes, intermediate sizes
  int64_t cd[RTR_MAX_ORDER];
  for (int n = 0; n < order; ++n) cd[n] = dims[n];
  size_t pmax = 0, midmax = 0;
  int last = -1;
  bool first = true;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    if (k == dims[n]) continue;
    rtr::ModeView v = mode_view(cd, order, n);
    const rtr::Arith an = first ? ar : rtr::kF64;
    const int kb = rtr::fast_pass_block_k(an, v, (int)k, 0);
    size_t need;
    if (kb > 0) {
      need = 0;
      const int64_t rb = row_block(v.In);
      for (int64_t r0 = 0; r0 < v.In; r0 += rb) {
        const int64_t rows = std::min(rb, v.In - r0);
        need = std::max(need, (size_t)rtr::fast_pass_grid(an, v, kb, 0, X, r0, rows) * rows * kb *
                                  sizeof(float));
      }
    } else {
      if (k > 64)
        return fail(h, RTR_ERR_UNSUPPORTED, "the sequential sketch takes K_n <= 64 past the first "
                                            "projected mode (mode " + std::to_string(n) + ")");
      need = (size_t)rtr::sketch_chunks(v, (int)k) * v.In * k *
             (an == rtr::kF64 ? sizeof(double) : sizeof(float));
    }
    pmax = std::max(pmax, need);
    cd[n] = k;
    size_t z = 1;
    for (int m = 0; m < order; ++m) z *= (size_t)cd[m];
    midmax = std::max(midmax, z);
    last = n;
    first = false;
  }
  Carve plan(nullptr);
  plan.take<char>(pmax);
  plan.take<double>(midmax);
  plan.take<double>(midmax);
  for (int n = 0; n < order; ++n) {
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
    plan.take<double>((size_t)dims[n] * keff(dims, K, n));
  }
  plan.take<double>(1024);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  void* partial = cv.take<char>(pmax);
  double* buf[2] = {cv.take<double>(midmax), cv.take<double>(midmax)};
  double* Ycol[RTR_MAX_ORDER];
  double* Qw[RTR_MAX_ORDER];
  double* Qn[RTR_MAX_ORDER];
  size_t qoff = 0;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    Ycol[n] = cv.take<double>((size_t)dims[n] * k);
    Qw[n] = cv.take<double>((size_t)dims[n] * k);
    Qn[n] = Q + qoff;
    qoff += (size_t)dims[n] * k;
  }
  double* red = cv.take<double>(1024);

  for (int n = 0; n < order; ++n) cd[n] = dims[n];
  const void* cur = X;
  bool cur_is_x = true;
  int nb = 0;
  for (int n = 0; n < order; ++n) {
    const int64_t k = keff(dims, K, n);
    if (k == dims[n]) {
      HIP_TRY(rtr::launch_identity(Qn[n], dims[n], s), "identity");
      continue;
    }
    rtr::ModeView v = mode_view(cd, order, n);
    const rtr::Arith an = cur_is_x ? ar : rtr::kF64;
    const int kmax = rtr::fast_pass_block_k(an, v, (int)k, 0);
    if (kmax > 0) {
      const int64_t rb = row_block(v.In);
      for (int64_t r0 = 0; r0 < v.In; r0 += rb) {
        const int64_t rows = std::min(rb, v.In - r0);
        for (int k0 = 0; k0 < (int)k; k0 += kmax) {
          const int kb = std::min(kmax, (int)k - k0);
          const int64_t grid = rtr::fast_pass_grid(an, v, kb, 0, cur, r0, rows);
          HIP_TRY(rtr::launch_fast_pass(an, 0, cur, v, kb, seed, rtr::omega_stream(n), tensor_id,
                                        nullptr, partial, grid, s, r0, rows, (int)k, k0),
                  "sketch_fused");
          HIP_TRY(rtr::launch_reduce_partials(rtr::kF32, partial, grid, rows, kb,
                                              Ycol[n] + (int64_t)k0 * v.In + r0, s, v.In),
                  "reduce_partials");
        }
      }
    } else {
      const int64_t chunks = rtr::sketch_chunks(v, (int)k);
      HIP_TRY(rtr::launch_sketch_partial(an, cur, v, (int)k, seed, rtr::omega_stream(n), tensor_id,
                                         partial, chunks, s),
              "sketch_partial");
      HIP_TRY(rtr::launch_reduce_partials(an, partial, chunks, v.In, (int)k, Ycol[n], s),
              "reduce_partials");
    }
    rtr::QrJobs jobs{};
    jobs.count = 1;
    jobs.A[0] = Ycol[n];
    jobs.Qwork[0] = Qw[n];
    jobs.In[0] = dims[n];
    jobs.K[0] = (int)k;
    jobs.Q[0] = Qn[n];
    HIP_TRY(rtr::launch_householder_qr(jobs, s), "householder_qr");
    double* out = (n == last) ? P : buf[nb];
    HIP_TRY(rtr::launch_ttm(not_fp8(ar), cur_is_x, cur, v, (int)k, Qn[n], out, s), "ttm");
    cd[n] = k;
    cur = out;
    cur_is_x = false;
    nb ^= 1;
  }
  if (last < 0) {  // nothing projected: P = X in FP64 (the product with Q_1 = I)
    rtr::ModeView v = mode_view(dims, order, 0);
    HIP_TRY(rtr::launch_ttm(not_fp8(ar), true, X, v, (int)dims[0], Qn[0], P, s), "ttm");
  }
  if (p_norm2) HIP_TRY(rtr::launch_sumsq(false, P, (int64_t)pnum, red, p_norm2, s), "sumsq");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_decompose(rtr_handle h, const double* P, int32_t order, const int32_t* Kp,
                         const int32_t* R, const rtr_decompose_opts* opts,
                         const double* Z_init, double* Z, double* err_trace,
                         int32_t* sweeps_run, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (!opts) return fail(h, RTR_ERR_INVALID_ARG, "opts is NULL");
  if (opts->method == RTR_METHOD_SVD)
    return fail(h, RTR_ERR_INVALID_ARG, "TR-SVD chooses the ranks: call rtr_decompose_svd");
  if (opts->method != RTR_METHOD_ALS) return fail(h, RTR_ERR_INVALID_ARG, "unknown method");
  if (order < 2 || order > RTR_MAX_ORDER)
    return fail(h, RTR_ERR_INVALID_ARG, "decomposition needs 2 <= order <= 8");
  if (!Kp || !R) return fail(h, RTR_ERR_INVALID_ARG, "Kp and R must be host arrays");
  if (!P || !Z_init || !Z || !err_trace || !sweeps_run)
    return fail(h, RTR_ERR_INVALID_ARG, "P, Z_init, Z, err_trace, sweeps_run must be device pointers");
  if (opts->max_sweeps < 1) return fail(h, RTR_ERR_INVALID_ARG, "max_sweeps must be >= 1");
  if (!(opts->tol >= 0.0)) return fail(h, RTR_ERR_INVALID_ARG, "tol must be >= 0");
  int64_t total = 1;
  for (int n = 0; n < order; ++n) {
    if (Kp[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, "Kp entries must be >= 1");
    if (R[n] < 1 || R[n] > RTR_MAX_RANK)
      return fail(h, RTR_ERR_INVALID_ARG, "ranks must be in [1, " + std::to_string(RTR_MAX_RANK) + "]");
    total *= Kp[n];
  }
  hipStream_t s = (hipStream_t)stream;
  size_t zoff[RTR_MAX_ORDER + 1];
  zoff[0] = 0;
  int64_t Jmax = 0;
  int RRmax = 0, noutmax = 0;
  int64_t chunkmax = 1;
  rtr::AlsGeom geo[RTR_MAX_ORDER];
  int64_t strideP[RTR_MAX_ORDER];
  strideP[order - 1] = 1;
  for (int n = order - 2; n >= 0; --n) strideP[n] = strideP[n + 1] * Kp[n + 1];
  for (int n = 0; n < order; ++n) {
    const int Ra = R[n], Rb = R[(n + 1) % order];
    zoff[n + 1] = zoff[n] + (size_t)Ra * Kp[n] * Rb;
    rtr::AlsGeom g{};
    g.N = order;
    g.n = n;
    g.Kn = Kp[n];
    g.Ra = Ra;
    g.Rb = Rb;
    g.RR = Ra * Rb;
    g.J = total / Kp[n];
    for (int t = 1; t < order; ++t) {
      const int m = (n + t) % order;
      g.cycK[t - 1] = Kp[m];
      g.cycStride[t - 1] = strideP[m];
    }
    g.strideN = strideP[n];
    if ((int64_t)g.RR > g.J)
      return fail(h, RTR_ERR_INVALID_ARG,
                  "R_n R_{n+1} exceeds the number of equations for core " + std::to_string(n));
    if (!rtr::als_supported(g.Kn, g.RR))
      return fail(h, RTR_ERR_UNSUPPORTED, "TR-ALS takes K'_n <= 1024 and R_n R_{n+1} <= 256");
    geo[n] = g;
    Jmax = std::max(Jmax, g.J);
    RRmax = std::max(RRmax, g.RR);
    noutmax = std::max(noutmax, g.Kn * g.RR + g.RR * g.RR);
    chunkmax = std::max(chunkmax, rtr::als_chunks(g));
  }
  CHECK_DEV(P, (size_t)total * sizeof(double), "P");
  CHECK_DEV(Z_init, zoff[order] * sizeof(double), "Z_init");
  CHECK_DEV(Z, zoff[order] * sizeof(double), "Z");
  CHECK_DEV(err_trace, (size_t)opts->max_sweeps * sizeof(double), "err_trace");
  CHECK_DEV(sweeps_run, sizeof(int32_t), "sweeps_run");
  if (h->als_launch == 0) {  // the whole decomposition in one cooperative launch
    rtr::AlsPersistArgs pa{};
    pa.N = order;
    for (int n = 0; n < order; ++n) {
      pa.K[n] = Kp[n];
      pa.R[n] = R[n];
      pa.zoff[n] = (int64_t)zoff[n];
      pa.strideP[n] = strideP[n];
    }
    pa.total = total;
    pa.ztotal = (int64_t)zoff[order];
    size_t plds = 0;
    if (rtr::als_persist_plan(&pa, &plds)) {
      Carve plan(nullptr);
      plan.take<double>((size_t)pa.G * pa.rec);
      plan.take<double>((size_t)pa.rec);
      plan.take<double>(1024);
      plan.take<double>(1);
      plan.take<unsigned>(1);
      if ((st = ensure_ws(h, plan.off + 256))) return st;
      Carve cv(h->ws);
      pa.part = cv.take<double>((size_t)pa.G * pa.rec);
      pa.red = cv.take<double>((size_t)pa.rec);
      double* red = cv.take<double>(1024);
      double* pn2 = cv.take<double>(1);
      pa.bar = cv.take<unsigned>(1);
      if (Z != Z_init)
        HIP_TRY(hipMemcpyAsync(Z, Z_init, zoff[order] * sizeof(double), hipMemcpyDeviceToDevice, s),
                "hipMemcpyAsync");
      HIP_TRY(rtr::launch_sumsq(false, P, total, red, pn2, s), "sumsq");
      pa.P = P;
      pa.Z = Z;
      pa.pn2 = pn2;
      pa.status = h->status;
      pa.trace = err_trace;
      pa.sweeps_run = sweeps_run;
      pa.tol = opts->tol;
      pa.max_sweeps = opts->max_sweeps;
      pa.spin_limit = 1u << 22;
      const hipError_t e = rtr::launch_als_persist(pa, plds, s);
      if (e == hipSuccess) return RTR_OK;
      if (e != hipErrorCooperativeLaunchTooLarge) return hip_fail(h, e, "single-launch TR-ALS");
      (void)hipGetLastError();  // not enough co-resident work-groups: per-update launches
    }
  }
  int rmax = 0;
  for (int n = 0; n < order; ++n) rmax = std::max(rmax, (int)R[n]);
  // Gram from transfer matrices when every rank is at most 7 and the cores fit the solve's
  // LDS staging; otherwise accumulated directly as B^T B
  int maxK = 0;
  for (int n = 0; n < order; ++n) maxK = std::max(maxK, (int)Kp[n]);
  const int gram_direct = (rmax > 7 || zoff[order] > 6144 || maxK > 64) ? 1 : 0;
  const int tdim = rtr::als2_tdim(rmax);
  bool use2 = total < (1LL << 31);
  int64_t grid2max = 1;
  for (int n = 0; n < order; ++n) {
    use2 = use2 && rtr::als2_supported(geo[n].Kn, geo[n].RR, geo[n].J, (int64_t)zoff[order],
                                       gram_direct, tdim, maxK);
    grid2max = std::max(grid2max, rtr::als2_parts(geo[n].Kn, geo[n].RR, geo[n].J,
                                                  (int64_t)zoff[order]));
  }
  Carve plan(nullptr);
  plan.take<double>((size_t)Jmax * RRmax);
  plan.take<double>((size_t)std::max(chunkmax, grid2max) * (noutmax + 1));
  plan.take<double>(noutmax);
  plan.take<double>(chunkmax);
  plan.take<double>(1024);
  plan.take<double>(1);
  plan.take<int>(1);
  plan.take<double>((size_t)RRmax * RRmax);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  double* Bm = cv.take<double>((size_t)Jmax * RRmax);
  double* part = cv.take<double>((size_t)std::max(chunkmax, grid2max) * (noutmax + 1));
  double* MG = cv.take<double>(noutmax);
  double* rpart = cv.take<double>(chunkmax);
  double* red = cv.take<double>(1024);
  double* pn2 = cv.take<double>(1);
  int* done = cv.take<int>(1);
  double* gram = cv.take<double>((size_t)RRmax * RRmax);  // transfer-matrix Gram of the update

  if (Z != Z_init)
    HIP_TRY(hipMemcpyAsync(Z, Z_init, zoff[order] * sizeof(double), hipMemcpyDeviceToDevice, s),
            "hipMemcpyAsync");
  HIP_TRY(rtr::launch_sumsq(false, P, total, red, pn2, s), "sumsq");
  HIP_TRY(rtr::launch_als_begin(done, sweeps_run, s), "als_begin");
  if (use2) {
    auto args_for = [&](int n, int mode) {
      const rtr::AlsGeom& g = geo[n];
      rtr::AlsArgs2 a{};
      a.P = P;
      a.Z = Z;
      a.N = order;
      a.n = n;
      a.Kn = g.Kn;
      a.Ra = g.Ra;
      a.Rb = g.Rb;
      a.RR = g.RR;
      a.J = g.J;
      for (int t = 0; t < order - 1; ++t) {
        const int m = (n + 1 + t) % order;
        a.cycK[t] = g.cycK[t];
        a.cycStride[t] = g.cycStride[t];
        a.chI[t] = Kp[m];
        a.chRb[t] = R[(m + 1) % order];
        a.chOff[t] = (int64_t)zoff[m];
      }
      a.strideN = g.strideN;
      a.zoffN = (int64_t)zoff[n];
      a.mode = mode;
      a.gram_direct = gram_direct;
      a.ztotal = (int64_t)zoff[order];
      a.part = part;
      a.done = done;
      // the transfer-matrix Gram of core n is formed by one extra work-group of this launch
      a.gram_extra = (!gram_direct && (mode & 1)) ? 1 : 0;
      a.gram_out = gram;
      a.tdim = tdim;
      for (int m = 0; m < order; ++m) {
        a.zoffs[m] = (int64_t)zoff[m];
        a.Kc[m] = Kp[m];
        a.Rc[m] = R[m];
      }
      return a;
    };
    auto solve_for = [&](int n, int64_t grid, int report, int report_only) {
      const rtr::AlsGeom& g = geo[n];
      rtr::AlsSolveArgs a{};
      a.part = part;
      a.red = MG;
      a.nparts = (int)grid;
      a.Kn = g.Kn;
      a.RR = g.RR;
      a.Rb = g.Rb;
      a.Ra = g.Ra;
      a.gram_direct = gram_direct;
      a.N = order;
      a.n = n;
      a.Z = Z;
      for (int m = 0; m < order; ++m) {
        a.zoff[m] = (int64_t)zoff[m];
        a.Kc[m] = Kp[m];
        a.Rc[m] = R[m];
      }
      a.tdim = tdim;
      a.ztotal = (int64_t)zoff[order];
      a.Zn = Z + zoff[n];
      a.status = h->status;
      a.done = done;
      a.report_sweep = report;
      a.report_only = report_only;
      a.pn2 = pn2;
      a.trace = err_trace;
      a.sweeps_run = sweeps_run;
      a.tol = opts->tol;
      a.gram_in = (!gram_direct && !report_only) ? gram : nullptr;
      return a;
    };
    for (int sw = 0; sw < opts->max_sweeps; ++sw) {
      for (int n = 0; n < order; ++n) {
        const bool rep = (n == 0 && sw > 0);
        const int64_t grid = rtr::als2_parts(geo[n].Kn, geo[n].RR, geo[n].J, (int64_t)zoff[order]);
        HIP_TRY(rtr::launch_als_accum(args_for(n, 1 | (rep ? 2 : 0)), rmax, s), "als_accum");
        HIP_TRY(rtr::launch_als_solve2(solve_for(n, grid, rep ? sw - 1 : -1, 0), s), "als_solve");
      }
    }
    const int64_t grid = rtr::als2_parts(geo[0].Kn, geo[0].RR, geo[0].J, (int64_t)zoff[order]);
    HIP_TRY(rtr::launch_als_accum(args_for(0, 2), rmax, s), "als_accum");
    HIP_TRY(rtr::launch_als_solve2(solve_for(0, grid, opts->max_sweeps - 1, 1), s), "als_solve");
    return RTR_OK;
  }
  for (int sw = 0; sw < opts->max_sweeps; ++sw) {
    for (int n = 0; n < order; ++n) {
      const rtr::AlsGeom& g = geo[n];
      rtr::Chain ch{};
      ch.L = order - 1;
      for (int t = 1; t < order; ++t) {
        const int m = (n + t) % order;
        ch.core[t - 1] = Z + zoff[m];
        ch.I[t - 1] = Kp[m];
        ch.Ra[t - 1] = R[m];
        ch.Rb[t - 1] = R[(m + 1) % order];
      }
      HIP_TRY(rtr::launch_chain(ch, g.J, 1, Bm, done, s), "chain");
      const int64_t chunks = rtr::als_chunks(g);
      const int nout = g.Kn * g.RR + g.RR * g.RR;
      HIP_TRY(rtr::launch_als_partial(P, g, Bm, part, chunks, done, s), "als_partial");
      HIP_TRY(rtr::launch_als_reduce(part, chunks, nout, MG, done, s), "als_reduce");
      HIP_TRY(rtr::launch_als_solve(MG, g, Z + zoff[n], h->status, done, s), "als_solve");
      if (n == order - 1) {
        HIP_TRY(rtr::launch_als_resid(P, g, Bm, Z + zoff[n], rpart, chunks, done, s), "als_resid");
        HIP_TRY(rtr::launch_als_err(rpart, chunks, pn2, sw, opts->tol, err_trace, sweeps_run, done, s),
                "als_err");
      }
    }
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_decompose_svd(rtr_handle h, const double* P, int32_t order, const int32_t* Kp,
                             const int32_t* Rcap, double eps, double* Z, int32_t* ranks,
                             double* err, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (order < 2 || order > RTR_MAX_ORDER)
    return fail(h, RTR_ERR_INVALID_ARG, "decomposition needs 2 <= order <= 8");
  if (!Kp || !Rcap) return fail(h, RTR_ERR_INVALID_ARG, "Kp and Rcap must be host arrays");
  if (!P || !Z || !ranks || !err)
    return fail(h, RTR_ERR_INVALID_ARG, "P, Z, ranks, err must be device pointers");
  if (!(eps > 0.0) || !(eps < 1e300)) return fail(h, RTR_ERR_INVALID_ARG, "eps must be > 0");
  int64_t total = 1;
  for (int n = 0; n < order; ++n) {
    if (Kp[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, "Kp entries must be >= 1");
    if (Rcap[n] < 1 || Rcap[n] > rtr::kSvdMaxDim)
      return fail(h, RTR_ERR_INVALID_ARG, "rank caps must be in [1, 512]");
    total *= Kp[n];
    if (total > ((int64_t)1 << 31)) return fail(h, RTR_ERR_UNSUPPORTED, "P above 2^31 entries");
  }
  {
    size_t zb = 0;
    for (int n = 0; n < order; ++n) zb += (size_t)Rcap[n] * Kp[n] * Rcap[(n + 1) % order];
    CHECK_DEV(P, (size_t)total * sizeof(double), "P");
    CHECK_DEV(Z, zb * sizeof(double), "Z");
    CHECK_DEV(ranks, (size_t)order * sizeof(int32_t), "ranks");
    CHECK_DEV(err, sizeof(double), "err");
  }
  // Bounds of the Gram sizes: step 0 has d_0 = min(K_1, prod K / K_1); R_1 <= R_2 and
  // R_1 R_2 <= d_0; step k >= 1 works on (R_{k+1} K_k) x (K_{k+1} .. K_N R_1) with
  // R_{k+1} <= min(cap, d_{k-1}).
  int dmax[RTR_MAX_ORDER];
  int dall = 0;
  int64_t rb[RTR_MAX_ORDER];
  for (int k = 0; k + 1 < order; ++k) {
    int64_t rest = 1;
    for (int j = k + 1; j < order; ++j) rest *= Kp[j];
    int64_t d;
    if (k == 0) {
      d = std::min((int64_t)Kp[0], rest);
      int64_t sq = 1;
      while ((sq + 1) * (sq + 1) <= d) ++sq;
      rb[0] = std::min((int64_t)Rcap[0], sq);
      rb[1] = std::min((int64_t)Rcap[1], d);
    } else {
      d = std::min(rb[k] * Kp[k], rest * rb[0]);
      if (k + 1 < order) rb[k + 1] = std::min((int64_t)Rcap[k + 1], d);
    }
    if (d > rtr::kSvdMaxDim)
      return fail(h, RTR_ERR_UNSUPPORTED,
                  "TR-SVD step " + std::to_string(k) + " may need a Gram of size " +
                      std::to_string(d) + " > 512 (lower the rank caps)");
    dmax[k] = (int)d;
    dall = std::max(dall, (int)d);
  }
  hipStream_t s = (hipStream_t)stream;
  Carve plan(nullptr);
  plan.take<double>(1024);
  plan.take<double>(1);
  plan.take<rtr::SvdState>(1);
  plan.take<double>((size_t)dall * dall);
  plan.take<double>((size_t)dall * dall);
  plan.take<double>((size_t)dall * dall);
  plan.take<double>(dall);
  plan.take<double>(total);
  plan.take<double>(total);
  st = ensure_ws(h, plan.off);
  if (st) return st;
  Carve c(h->ws);
  double* red = c.take<double>(1024);
  double* pn2 = c.take<double>(1);
  rtr::SvdState* state = c.take<rtr::SvdState>(1);
  double* A = c.take<double>((size_t)dall * dall);
  double* V = c.take<double>((size_t)dall * dall);
  double* W = c.take<double>((size_t)dall * dall);
  double* sv = c.take<double>(dall);
  double* buf[2] = {c.take<double>(total), c.take<double>(total)};
  rtr::SvdCaps caps{};
  caps.N = order;
  for (int n = 0; n < order; ++n) caps.c[n] = Rcap[n];
  size_t slot[RTR_MAX_ORDER];
  slot[0] = 0;
  for (int n = 0; n + 1 < order; ++n)
    slot[n + 1] = slot[n] + (size_t)Rcap[n] * Kp[n] * Rcap[(n + 1) % order];
  HIP_TRY(rtr::launch_sumsq(false, P, total, red, pn2, s), "sumsq");
  HIP_TRY(rtr::launch_svd_init(state, pn2, eps, order, Kp[0], (int)(total / Kp[0]), s),
          "svd init");
  const double* C = P;
  for (int k = 0; k + 1 < order; ++k) {
    double* Cn = buf[k & 1];
    HIP_TRY(rtr::launch_svd_step(state, C, A, V, W, sv, caps, k, dmax[k], Z + slot[k], Cn,
                                 Kp[k + 1], s),
            "svd step");
    C = Cn;
  }
  HIP_TRY(rtr::launch_svd_last(state, C, Z + slot[order - 1], order, ranks, err, h->status, s),
          "svd last");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
namespace {

struct BatchPlan {
  std::vector<rtr::AlsItem> items;
  rtr::BatchLayout lay{};
  int mq = 1, gq = 4;
};

rtr_status plan_batch(rtr_context* h, const rtr_als_item* items, int32_t count,
                      int32_t max_sweeps, double tol, BatchPlan* plan) {
  if (!items || count < 1) return fail(h, RTR_ERR_INVALID_ARG, "items must hold count >= 1 entries");
  if (count > 65535) return fail(h, RTR_ERR_UNSUPPORTED, "at most 65535 tensors per batch");
  if (max_sweeps < 1) return fail(h, RTR_ERR_INVALID_ARG, "max_sweeps must be >= 1");
  if (!(tol >= 0.0)) return fail(h, RTR_ERR_INVALID_ARG, "tol must be >= 0");
  int maxK = 1, maxRR = 1, maxR = 1, minK = 1 << 30;
  int64_t maxZ = 1;
  plan->items.resize(count);
  for (int t = 0; t < count; ++t) {
    const rtr_als_item& it = items[t];
    const std::string where = "item " + std::to_string(t) + ": ";
    if (it.order < 2 || it.order > RTR_MAX_ORDER)
      return fail(h, RTR_ERR_INVALID_ARG, where + "order must be in [2, 8]");
    if (!it.P || !it.Z_init || !it.Z || !it.err_trace || !it.sweeps_run)
      return fail(h, RTR_ERR_INVALID_ARG, where + "P, Z_init, Z, err_trace, sweeps_run must be device pointers");
    rtr::AlsItem a{};
    a.P = it.P;
    a.Zinit = it.Z_init;
    a.Z = it.Z;
    a.err = it.err_trace;
    a.sweeps = it.sweeps_run;
    a.N = it.order;
    int64_t total = 1, ztot = 0;
    for (int n = 0; n < it.order; ++n) {
      if (it.Kp[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, where + "Kp entries must be >= 1");
      if (it.R[n] < 1) return fail(h, RTR_ERR_INVALID_ARG, where + "ranks must be >= 1");
      if (it.Kp[n] > 64 || it.R[n] > 6)
        return fail(h, RTR_ERR_UNSUPPORTED, where + "the batched TR-ALS takes K'_n <= 64 and R_n <= 6");
      total *= it.Kp[n];
      if (total > ((int64_t)1 << 31)) return fail(h, RTR_ERR_UNSUPPORTED, where + "P above 2^31 entries");
      a.K[n] = it.Kp[n];
      a.R[n] = it.R[n];
    }
    for (int n = 0; n < it.order; ++n) {
      const int rb = it.R[(n + 1) % it.order];
      if ((int64_t)it.R[n] * rb > total / it.Kp[n])
        return fail(h, RTR_ERR_INVALID_ARG, where + "R_n R_{n+1} exceeds the number of equations of core " + std::to_string(n));
      ztot += (int64_t)it.R[n] * it.Kp[n] * rb;
      maxK = std::max(maxK, (int)it.Kp[n]);
      minK = std::min(minK, (int)it.Kp[n]);
      maxR = std::max(maxR, (int)it.R[n]);
      maxRR = std::max(maxRR, (int)(it.R[n] * rb));
    }
    maxZ = std::max(maxZ, ztot);
    rtr_status sc;
    if ((sc = check_dev(h, it.P, (size_t)total * sizeof(double), (where + "P").c_str())) ||
        (sc = check_dev(h, it.Z_init, (size_t)ztot * sizeof(double), (where + "Z_init").c_str())) ||
        (sc = check_dev(h, it.Z, (size_t)ztot * sizeof(double), (where + "Z").c_str())) ||
        (sc = check_dev(h, it.err_trace, (size_t)max_sweeps * sizeof(double), (where + "err_trace").c_str())) ||
        (sc = check_dev(h, it.sweeps_run, sizeof(int32_t), (where + "sweeps_run").c_str())))
      return sc;
    plan->items[t] = a;
  }
  if (!rtr::batch_layout(maxK, maxRR, maxR, maxZ, minK, &plan->lay, &plan->mq, &plan->gq))
    return fail(h, RTR_ERR_UNSUPPORTED, "batch does not fit the work-group's LDS (cores too large)");
  return RTR_OK;
}

// Copy the item array to the device through pinned staging (stream-ordered).
rtr_status upload_items(rtr_context* h, const std::vector<rtr::AlsItem>& v, hipStream_t s,
                        rtr::AlsItem** out) {
  const size_t bytes = v.size() * sizeof(rtr::AlsItem);
  if (h->items_copied) HIP_TRY(hipEventSynchronize(h->items_copied), "hipEventSynchronize");
  else HIP_TRY(hipEventCreateWithFlags(&h->items_copied, hipEventDisableTiming), "hipEventCreate");
  if (bytes > h->host_cap) {
    if (h->items_host) (void)hipHostFree(h->items_host);
    h->items_host = nullptr;
    h->host_cap = 0;
    HIP_TRY(hipHostMalloc(&h->items_host, bytes, hipHostMallocDefault), "hipHostMalloc");
    h->host_cap = bytes;
  }
  if (bytes > h->items_cap) {
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (h->items_dev) (void)hipFree(h->items_dev);
    h->items_dev = nullptr;
    h->items_cap = 0;
    HIP_TRY(hipMalloc(&h->items_dev, bytes), "hipMalloc");
    h->items_cap = bytes;
  }
  std::memcpy(h->items_host, v.data(), bytes);
  HIP_TRY(hipMemcpyAsync(h->items_dev, h->items_host, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  HIP_TRY(hipEventRecord(h->items_copied, s), "hipEventRecord");
  *out = (rtr::AlsItem*)h->items_dev;
  return RTR_OK;
}

uint64_t fnv(uint64_t hsh, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) hsh = (hsh ^ b[i]) * 1099511628211ull;
  return hsh;
}

}  // namespace

rtr_status rtr_decompose_batch(rtr_handle h, const rtr_als_item* items, int32_t count,
                               int32_t max_sweeps, double tol, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  BatchPlan plan;
  st = plan_batch(h, items, count, max_sweeps, tol, &plan);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  rtr::AlsItem* dev = nullptr;
  st = upload_items(h, plan.items, s, &dev);
  if (st) return st;
  HIP_TRY(rtr::launch_als_batch(dev, count, max_sweeps, tol, h->status, plan.lay, plan.mq, plan.gq, s),
          "batched TR-ALS");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

namespace {

// Alg. 1 steps 3-12 for every item: per-tensor sketch and compression, one batched TR-ALS
// launch over the item array ``dev``, per-tensor back-projection.
// ---------------------------------------------------------------------------------------
// Batched work lists: the sketches of every (tensor, mode) in one launch, their sums in one,
// every QR in one, and each mode product of the compression chain (mode 1 first, Eq. 3) for
// every tensor in one launch per mode.  The job arrays hold device addresses inside the
// workspace, so they are built and uploaded once per call, before the eager run and the
// capture, and reused by both.
struct StreamPlan {
  rtr::Arith ar = rtr::kF32;
  int kc = 16;
  int njobs = 0;
  int64_t sk_blocks = 0, sk_maxout = 0;
  const rtr::SketchJob* d_sk = nullptr;
  const int64_t* d_skstart = nullptr;
  double* const* d_work = nullptr;
  double* const* d_qout = nullptr;
  std::vector<std::pair<double*, int64_t>> ident;  // modes kept: Q_n = I
  int steps = 0;
  std::vector<int> tt_n;
  std::vector<int64_t> tt_blocks;
  std::vector<const rtr::TtmJob*> d_tt;
  std::vector<const int64_t*> d_ttstart;
};

// The work lists of the batched path.  (They were once switched off after a GPU memory fault in
// the first graph-captured run; the cause was a stray release of the job arrays before the
// capture, which left the captured launches reading freed memory.)
constexpr bool kBatchWorkLists = true;

bool stream_eligible(const rtr_batch_item* items, int32_t count, rtr_dtype x_dtype,
                     int32_t power_iters) {
  if (!kBatchWorkLists) return false;
  if (x_dtype != RTR_F32 || power_iters != 0) return false;
  for (int t = 0; t < count; ++t)
    for (int n = 0; n < items[t].order; ++n)
      if (keff(items[t].dims, items[t].K, n) > 64) return false;
  return true;
}

rtr_status plan_stream(rtr_context* h, const rtr_batch_item* items, int32_t count, rtr::Arith ar,
                       int target, int kc, hipStream_t s, StreamPlan* sp) {
  sp->ar = ar;
  sp->kc = kc;
  int maxorder = 0;
  for (int t = 0; t < count; ++t) maxorder = std::max(maxorder, (int)items[t].order);
  // sizes: sketch partials, Ycol + Qwork per job, two intermediates per tensor
  size_t part = 0, yq = 0, mid = 0;
  int njobs = 0;
  std::vector<size_t> midt(count, 0);
  for (int t = 0; t < count; ++t) {
    const rtr_batch_item& it = items[t];
    int64_t cur[RTR_MAX_ORDER];
    for (int n = 0; n < it.order; ++n) cur[n] = it.dims[n];
    for (int n = 0; n < it.order; ++n) {
      const int64_t k = keff(it.dims, it.K, n);
      if (k < it.dims[n]) {
        rtr::ModeView v = mode_view(it.dims, it.order, n);
        part += (size_t)rtr::sketch_job_chunks(v, (int)k, target) * v.In * k;
        yq += 2 * (size_t)v.In * k;
        ++njobs;
      }
      cur[n] = k;
      if (n + 1 < it.order) {
        size_t z = 1;
        for (int m = 0; m < it.order; ++m) z *= (size_t)cur[m];
        midt[t] = std::max(midt[t], z);
      }
    }
    mid += 2 * midt[t];
  }
  Carve plan(nullptr);
  plan.take<float>(part);
  plan.take<double>(yq);
  plan.take<double>(mid);
  rtr_status st;
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  float* pbase = cv.take<float>(part);
  double* ybase = cv.take<double>(yq);
  double* mbase = cv.take<double>(mid);
  // host job arrays
  std::vector<rtr::SketchJob> sk;
  std::vector<int64_t> skstart(1, 0);
  std::vector<double*> work, qout;
  std::vector<std::vector<rtr::TtmJob>> tt(maxorder);
  std::vector<std::vector<int64_t>> ttstart(maxorder, std::vector<int64_t>(1, 0));
  sp->ident.clear();
  size_t po = 0, yo = 0, mo = 0;
  for (int t = 0; t < count; ++t) {
    const rtr_batch_item& it = items[t];
    double* buf[2] = {mbase + mo, mbase + mo + midt[t]};
    mo += 2 * midt[t];
    size_t qoff = 0;
    int64_t cur[RTR_MAX_ORDER];
    for (int n = 0; n < it.order; ++n) cur[n] = it.dims[n];
    const void* in = it.X;
    for (int n = 0; n < it.order; ++n) {
      const int64_t k = keff(it.dims, it.K, n);
      double* Qn = it.Q + qoff;
      qoff += (size_t)it.dims[n] * k;
      rtr::ModeView v = mode_view(it.dims, it.order, n);
      if (k < it.dims[n]) {
        rtr::SketchJob g{};
        const int64_t chunks = rtr::sketch_job_chunks(v, (int)k, target);
        rtr::sketch_job_fill(g, it.X, v, (int)k, it.seed, rtr::omega_stream(n), it.tensor_id, chunks,
                             pbase + po, ybase + yo);
        po += (size_t)chunks * v.In * k;
        work.push_back(ybase + yo + (size_t)v.In * k);
        qout.push_back(Qn);
        yo += 2 * (size_t)v.In * k;
        sk.push_back(g);
        skstart.push_back(skstart.back() + rtr::sketch_job_blocks(g));
        sp->sk_maxout = std::max(sp->sk_maxout, v.In * k);
      } else {
        sp->ident.push_back({Qn, it.dims[n]});
      }
      // mode product n of tensor t: cur -> cur with I_n replaced by K'_n
      rtr::ModeView cv2 = mode_view(cur, it.order, n);
      rtr::TtmJob tj{};
      tj.in = in;
      tj.A = cv2.A;
      tj.In = cv2.In;
      tj.B = cv2.B;
      tj.K = (int)k;
      tj.Q = Qn;
      tj.out = (n + 1 == it.order) ? it.P : buf[n & 1];
      tt[n].push_back(tj);
      ttstart[n].push_back(ttstart[n].back() + rtr::ttm_job_blocks(tj, kc));
      in = tj.out;
      cur[n] = k;
    }
  }
  sp->njobs = (int)sk.size();
  sp->sk_blocks = skstart.back();
  sp->steps = maxorder;
  // one device array for every job list (uploaded synchronously, outside any capture)
  Carve jp(nullptr);
  jp.take<rtr::SketchJob>(sk.size());
  jp.take<int64_t>(skstart.size());
  jp.take<double*>(work.size());
  jp.take<double*>(qout.size());
  for (int n = 0; n < maxorder; ++n) {
    jp.take<rtr::TtmJob>(tt[n].size());
    jp.take<int64_t>(ttstart[n].size());
  }
  if (jp.off > h->jobs_cap) {
    if (h->ws_locked) return fail(h, RTR_ERR_INTERNAL, "job lists grew inside a graph capture");
    if (h->jobs_dev) {
      HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
      (void)hipFree(h->jobs_dev);
      h->jobs_dev = nullptr;
      h->jobs_cap = 0;
      ++h->ws_epoch;  // cached graphs read the old job arrays
    }
    HIP_TRY(hipMalloc(&h->jobs_dev, jp.off + 256), "hipMalloc");
    h->jobs_cap = jp.off + 256;
  }
  std::vector<char> host(jp.off + 256);
  Carve hc(host.data()), dc(h->jobs_dev);
  auto put = [&](const void* src, size_t bytes, size_t cnt, size_t elem) {
    void* hd = hc.take<char>(cnt * elem);
    void* dd = dc.take<char>(cnt * elem);
    if (bytes) std::memcpy(hd, src, bytes);
    return dd;
  };
  sp->d_sk = (const rtr::SketchJob*)put(sk.data(), sk.size() * sizeof(rtr::SketchJob), sk.size(),
                                         sizeof(rtr::SketchJob));
  sp->d_skstart = (const int64_t*)put(skstart.data(), skstart.size() * 8, skstart.size(), 8);
  sp->d_work = (double* const*)put(work.data(), work.size() * sizeof(double*), work.size(),
                                   sizeof(double*));
  sp->d_qout = (double* const*)put(qout.data(), qout.size() * sizeof(double*), qout.size(),
                                   sizeof(double*));
  sp->tt_n.assign(maxorder, 0);
  sp->tt_blocks.assign(maxorder, 0);
  sp->d_tt.assign(maxorder, nullptr);
  sp->d_ttstart.assign(maxorder, nullptr);
  for (int n = 0; n < maxorder; ++n) {
    sp->tt_n[n] = (int)tt[n].size();
    sp->tt_blocks[n] = ttstart[n].back();
    sp->d_tt[n] = (const rtr::TtmJob*)put(tt[n].data(), tt[n].size() * sizeof(rtr::TtmJob),
                                          tt[n].size(), sizeof(rtr::TtmJob));
    sp->d_ttstart[n] = (const int64_t*)put(ttstart[n].data(), ttstart[n].size() * 8,
                                           ttstart[n].size(), 8);
  }
  HIP_TRY(hipMemcpyAsync(h->jobs_dev, host.data(), hc.off, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return RTR_OK;
}

// The launches of a planned batch: sketches, sums, QR, then one mode product per mode.
rtr_status launch_stream(rtr_context* h, const StreamPlan& sp, hipStream_t s, int only = 0) {
  if (only != 2) {
    for (const auto& id : sp.ident) HIP_TRY(rtr::launch_identity(id.first, id.second, s), "identity");
    HIP_TRY(rtr::launch_sketch_list(sp.ar, sp.d_sk, sp.d_skstart, sp.njobs, sp.sk_blocks,
                                    sp.sk_maxout, s),
            "sketch_list");
    HIP_TRY(rtr::launch_qr_list(sp.d_sk, sp.d_work, sp.d_qout, sp.njobs, s), "qr_list");
  }
  if (only != 1)
    for (int n = 0; n < sp.steps; ++n)
      HIP_TRY(rtr::launch_ttm_list(sp.ar, n == 0, sp.kc, sp.d_tt[n], sp.d_ttstart[n], sp.tt_n[n],
                                   sp.tt_blocks[n], s),
              "ttm_list");
  return RTR_OK;
}

rtr_status batch_sequence(rtr_context* h, const rtr_batch_item* items, int32_t count,
                          rtr_dtype x_dtype, rtr_dtype compute, int32_t power_iters,
                          int32_t max_sweeps, double tol, const BatchPlan& plan,
                          const rtr::AlsItem* dev, hipStream_t s, int nb = 1,
                          const StreamPlan* sp = nullptr) {
  // Sketch and compression of every tensor.  With nb > 1 (graph capture only) tensor t goes
  // to branch stream t % nb with its own slice of the workspace, so that the launches of small
  // tensors, which leave most of the chip idle, overlap; the branches join before TR-ALS.
  char* const base = (char*)h->ws;
  const size_t cap = h->ws_cap;
  const size_t slice = nb > 1 ? (cap / nb) & ~size_t(255) : cap;
  if (nb > 1) {
    HIP_TRY(hipEventRecord(h->fork_ev, s), "hipEventRecord");
    for (int b = 0; b < nb; ++b) HIP_TRY(hipStreamWaitEvent(h->br[b], h->fork_ev, 0), "hipStreamWaitEvent");
    h->ws_locked = true;
  }
  rtr_status st = RTR_OK;
  if (sp) {
    Guard guard(h);
    st = launch_stream(h, *sp, s);
  }
  for (int t = 0; t < count && !st && !sp; ++t) {
    const rtr_batch_item& it = items[t];
    hipStream_t ts = nb > 1 ? h->br[t % nb] : s;
    if (nb > 1) {
      h->ws = base + (size_t)(t % nb) * slice;
      h->ws_cap = slice;
    }
    st = rtr_sketch(h, it.X, x_dtype, it.order, it.dims, it.K, power_iters, it.seed,
                    it.tensor_id, compute, it.Q, ts);
    if (!st)
      st = rtr_compress(h, it.X, x_dtype, it.order, it.dims, it.K, it.Q, compute, it.P, nullptr, ts);
  }
  if (nb > 1) {
    h->ws = base;
    h->ws_cap = cap;
    h->ws_locked = false;
    for (int b = 0; b < nb; ++b) {  // join every branch, also after an error
      HIP_TRY(hipEventRecord(h->join_ev[b], h->br[b]), "hipEventRecord");
      HIP_TRY(hipStreamWaitEvent(s, h->join_ev[b], 0), "hipStreamWaitEvent");
    }
  }
  if (st) return st;
  Guard guard(h);
  HIP_TRY(rtr::launch_als_batch(dev, count, max_sweeps, tol, h->status, plan.lay, plan.mq, plan.gq, s),
          "batched TR-ALS");
  for (int t = 0; t < count; ++t) {
    const rtr_batch_item& it = items[t];
    if (!it.G) continue;
    rtr_status st = rtr_backproject(h, it.order, it.dims, it.K, it.R, it.Z, it.Q, it.G, s);
    if (st) return st;
  }
  return RTR_OK;
}

}  // namespace

rtr_status rtr_batch_autotune(rtr_handle h, const rtr_batch_item* items, int32_t count,
                              rtr_dtype x_dtype, rtr_dtype compute, int32_t* table,
                              void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  if (!items || count < 1 || !table) return fail(h, RTR_ERR_INVALID_ARG, "items, count, table");
  if (!kBatchWorkLists)
    return fail(h, RTR_ERR_UNSUPPORTED, "the batched work lists are switched off in this build");
  if (!stream_eligible(items, count, x_dtype, 0))
    return fail(h, RTR_ERR_UNSUPPORTED, "the batched work lists take FP32 X and K'_n <= 64");
  rtr::Arith ar;
  if ((st = check_arith(h, x_dtype, compute, &ar))) return st;
  ar = not_fp8(ar);
  for (int t = 0; t < count; ++t) {
    const rtr_batch_item& it = items[t];
    if (it.order < 2 || it.order > RTR_MAX_ORDER || !it.X || !it.Q || !it.P)
      return fail(h, RTR_ERR_INVALID_ARG, "item " + std::to_string(t) + ": order, X, Q, P");
    const std::string where = "item " + std::to_string(t) + ": ";
    rtr_status sc;
    if ((sc = check_dev(h, it.X, x_bytes(it.dims, it.order, x_dtype), (where + "X").c_str())) ||
        (sc = check_dev(h, it.Q, q_bytes(it.dims, it.K, it.order), (where + "Q").c_str())))
      return sc;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  // mean time of ``reps`` runs of one part of the work lists (after one untimed run)
  auto clock = [&](const StreamPlan& sp, int part, float* us) -> rtr_status {
    rtr_status r;
    if ((r = launch_stream(h, sp, s, part))) return r;
    HIP_TRY(hipEventRecord(e0, s), "hipEventRecord");
    for (int i = 0; i < 3; ++i)
      if ((r = launch_stream(h, sp, s, part))) return r;
    HIP_TRY(hipEventRecord(e1, s), "hipEventRecord");
    HIP_TRY(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    *us = ms * 1e3f / 3.f;
    return RTR_OK;
  };
  const int targets[3] = {16, 64, 256}, kcs[3] = {4, 16, 64};
  float tt[3], tk[3];
  int best_t = 0, best_k = 0;
  Guard guard(h);
  for (int i = 0; i < 3; ++i) {
    StreamPlan sp;
    if ((st = plan_stream(h, items, count, ar, targets[i], 16, s, &sp))) break;
    if ((st = clock(sp, 1, &tt[i]))) break;
    if (tt[i] < tt[best_t]) best_t = i;
  }
  for (int i = 0; i < 3 && !st; ++i) {
    StreamPlan sp;
    if ((st = plan_stream(h, items, count, ar, targets[best_t], kcs[i], s, &sp))) break;
    if ((st = clock(sp, 2, &tk[i]))) break;
    if (tk[i] < tk[best_k]) best_k = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  h->bt_target = targets[best_t];
  h->bt_kc = kcs[best_k];
  table[0] = h->bt_target;
  table[1] = h->bt_kc;
  for (int i = 0; i < 3; ++i) {
    table[2 + i] = (int32_t)(tt[i] + 0.5f);
    table[5 + i] = (int32_t)(tk[i] + 0.5f);
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_batch_run(rtr_handle h, const rtr_batch_item* items, int32_t count,
                         rtr_dtype x_dtype, rtr_dtype compute, int32_t power_iters,
                         int32_t max_sweeps, double tol, int32_t use_graph, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  if (!items || count < 1) return fail(h, RTR_ERR_INVALID_ARG, "items must hold count >= 1 entries");
  hipStream_t s = (hipStream_t)stream;
  // A call identical to the captured one (same item array and parameters) replays the graph;
  // its arguments were validated when it was captured.
  uint64_t key = 1469598103934665603ull;
  key = fnv(key, items, sizeof(rtr_batch_item) * (size_t)count);
  const int64_t params[7] = {count, x_dtype, compute, power_iters, max_sweeps, h->bt_target, h->bt_kc};
  key = fnv(key, params, sizeof(params));
  key = fnv(key, &tol, sizeof(tol));
  if (use_graph && h->gexec && key == h->gkey && h->gepoch == h->ws_epoch) {
    HIP_TRY(hipGraphLaunch(h->gexec, s), "hipGraphLaunch");
    return RTR_OK;
  }
  std::vector<rtr_als_item> als(count);
  for (int t = 0; t < count; ++t) {
    const rtr_batch_item& it = items[t];
    if (it.order < 2 || it.order > RTR_MAX_ORDER)
      return fail(h, RTR_ERR_INVALID_ARG, "item " + std::to_string(t) + ": order must be in [2, 8]");
    if (!it.X || !it.Q || !it.P)
      return fail(h, RTR_ERR_INVALID_ARG, "item " + std::to_string(t) + ": X, Q, P must be device pointers");
    rtr_als_item a{};
    a.P = it.P;
    a.Z_init = it.Z_init;
    a.Z = it.Z;
    a.err_trace = it.err_trace;
    a.sweeps_run = it.sweeps_run;
    a.order = it.order;
    for (int n = 0; n < it.order; ++n) {
      if (it.dims[n] < 1 || it.K[n] < 1)
        return fail(h, RTR_ERR_INVALID_ARG, "item " + std::to_string(t) + ": dims and K must be >= 1");
      a.Kp[n] = (int32_t)keff(it.dims, it.K, n);
      a.R[n] = it.R[n];
    }
    if (x_dtype != RTR_F64 && x_dtype != RTR_F32)
      return fail(h, RTR_ERR_UNSUPPORTED, "X must be FP64 or FP32");
    const std::string where = "item " + std::to_string(t) + ": ";
    size_t gb = 0;
    for (int n = 0; n < it.order; ++n)
      gb += (size_t)std::max(it.R[n], 1) * it.dims[n] * std::max(it.R[(n + 1) % it.order], 1);
    rtr_status sc;
    if ((sc = check_dev(h, it.X, x_bytes(it.dims, it.order, x_dtype), (where + "X").c_str())) ||
        (sc = check_dev(h, it.Q, q_bytes(it.dims, it.K, it.order), (where + "Q").c_str())) ||
        (sc = check_dev_opt(h, it.G, gb * sizeof(double), (where + "G").c_str())))
      return sc;
    als[t] = a;
  }
  BatchPlan plan;
  {
    Guard guard(h);
    st = plan_batch(h, als.data(), count, max_sweeps, tol, &plan);
    if (st) return st;
  }
  // the work lists of every tensor's sketch and compression, where the batch allows them
  StreamPlan splan;
  const bool streamed = h->bt_lists && stream_eligible(items, count, x_dtype, power_iters);
  rtr::Arith sar = rtr::kF32;
  if (streamed) {
    if ((st = check_arith(h, x_dtype, compute, &sar))) return st;
    sar = not_fp8(sar);
    Guard guard(h);
    if ((st = plan_stream(h, items, count, sar, h->bt_target, h->bt_kc, s, &splan))) return st;
  }
  const int splan_epoch = h->ws_epoch;  // the job lists point into this workspace
  // eager run (also sizes the workspace for the capture below)
  h->ws_hi = 0;
  rtr::AlsItem* dev = nullptr;
  {
    Guard guard(h);
    st = upload_items(h, plan.items, s, &dev);
    if (st) return st;
  }
  st = batch_sequence(h, items, count, x_dtype, compute, power_iters, max_sweeps, tol, plan, dev, s, 1,
                      streamed ? &splan : nullptr);
  if (st || !use_graph) return st;
  // capture the same sequence into a graph over a dedicated copy of the item array
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (streamed && h->ws_epoch != splan_epoch) {
    // the eager run grew the workspace: the job lists still point into the released one
    Guard guard(h);
    if ((st = plan_stream(h, items, count, sar, h->bt_target, h->bt_kc, s, &splan))) return st;
  }
  const size_t bytes = plan.items.size() * sizeof(rtr::AlsItem);
  if (bytes > h->gitems_cap) {
    if (h->gitems_dev) (void)hipFree(h->gitems_dev);
    h->gitems_dev = nullptr;
    h->gitems_cap = 0;
    HIP_TRY(hipMalloc(&h->gitems_dev, bytes), "hipMalloc");
    h->gitems_cap = bytes;
  }
  HIP_TRY(hipMemcpy(h->gitems_dev, plan.items.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
  const int nb = streamed ? 1 : std::min(kBatchBranches, count);
  if (nb > 1) {
    for (int b = 0; b < nb; ++b) {
      if (!h->br[b]) HIP_TRY(hipStreamCreateWithFlags(&h->br[b], hipStreamNonBlocking), "hipStreamCreate");
      if (!h->join_ev[b]) HIP_TRY(hipEventCreateWithFlags(&h->join_ev[b], hipEventDisableTiming), "hipEventCreate");
    }
    if (!h->fork_ev) HIP_TRY(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming), "hipEventCreate");
    // every branch gets a slice as large as the largest request of the eager run
    const size_t one = (h->ws_hi + 255) & ~size_t(255);
    {
      Guard guard(h);
      if ((st = ensure_ws(h, one * nb))) return st;
    }
  }
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  const int prof = h->prof_level;
  h->prof_level = 0;
  const int epoch = h->ws_epoch;
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
  st = batch_sequence(h, items, count, x_dtype, compute, power_iters, max_sweeps, tol, plan,
                      (const rtr::AlsItem*)h->gitems_dev, h->cap_stream, nb,
                      streamed ? &splan : nullptr);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
  h->prof_level = prof;
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return hip_fail(h, ec, "hipStreamEndCapture");
  if (h->ws_epoch != epoch) {
    (void)hipGraphDestroy(graph);
    return fail(h, RTR_ERR_INTERNAL, "workspace moved during graph capture");
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(h, ei, "hipGraphInstantiate");
  h->gexec = exec;
  h->gkey = key;
  h->gepoch = h->ws_epoch;
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
namespace {

rtr_status check_mlp(rtr_context* h, int32_t layers, const int32_t* sizes, int32_t batch,
                     rtr_dtype compute) {
  if (layers < 1 || layers > 16) return fail(h, RTR_ERR_INVALID_ARG, "layers must be in [1, 16]");
  if (!sizes) return fail(h, RTR_ERR_INVALID_ARG, "sizes is NULL");
  for (int l = 0; l <= layers; ++l)
    if (sizes[l] < 1) return fail(h, RTR_ERR_INVALID_ARG, "layer sizes must be >= 1");
  if (batch < 1) return fail(h, RTR_ERR_INVALID_ARG, "batch must be >= 1");
  if (compute != RTR_F32 && compute != RTR_BF16)
    return fail(h, RTR_ERR_UNSUPPORTED, "MLP compute must be RTR_F32 or RTR_BF16");
  return RTR_OK;
}

// Partial-sum workspace large enough for every product of one pass.
size_t gemm_ws_floats(int64_t M, int64_t N, int64_t K) {
  int64_t ks = 0;
  const int sl = rtr::gemm_slices(M, N, K, &ks);
  return (size_t)sl * M * N;
}

rtr_status run_gemm(rtr_context* h, bool bf, const float* A, int64_t sam, int64_t sak,
                    const float* B, int64_t sbk, int64_t sbn, int64_t M, int64_t N, int64_t K,
                    float* part, const float* bias, const float* mask, int mode, float* out,
                    hipStream_t s) {
  rtr::GemmArgs g{};
  g.A = A;
  g.B = B;
  g.part = part;
  g.M = M;
  g.N = N;
  g.K = K;
  g.sam = sam;
  g.sak = sak;
  g.sbk = sbk;
  g.sbn = sbn;
  const int sl = rtr::gemm_slices(M, N, K, &g.kslice);
  HIP_TRY(rtr::launch_gemm(bf, g, sl, s), "gemm");
  HIP_TRY(rtr::launch_epilogue(part, sl, M, N, bias, mask, mode, out, s), "gemm epilogue");
  return RTR_OK;
}

}  // namespace

rtr_status rtr_mlp_normalize(rtr_handle h, const double* P, int64_t dim, int32_t rows,
                             float* out, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (!P || !out || dim < 1 || rows < 1) return fail(h, RTR_ERR_INVALID_ARG, "bad arguments");
  CHECK_DEV(P, (size_t)dim * rows * sizeof(double), "P");
  CHECK_DEV(out, (size_t)dim * rows * sizeof(float), "out");
  HIP_TRY(rtr::launch_normalize(P, dim, rows, out, (hipStream_t)stream), "normalize");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_forward(rtr_handle h, int32_t layers, const int32_t* sizes,
                           const float* const* W, const float* const* b, const float* x,
                           int32_t batch, float* const* acts, float* y, rtr_dtype compute,
                           void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  st = check_mlp(h, layers, sizes, batch, compute);
  if (st) return st;
  if (!W || !b || !x || !y || (layers > 1 && !acts))
    return fail(h, RTR_ERR_INVALID_ARG, "W, b, x, y (and acts for hidden layers) required");
  CHECK_DEV(x, (size_t)batch * sizes[0] * sizeof(float), "x");
  CHECK_DEV(y, (size_t)batch * sizes[layers] * sizeof(float), "y");
  for (int l = 0; l < layers; ++l) {
    CHECK_DEV(W[l], (size_t)sizes[l] * sizes[l + 1] * sizeof(float), "W[l]");
    CHECK_DEV(b[l], (size_t)sizes[l + 1] * sizeof(float), "b[l]");
    if (l < layers - 1) CHECK_DEV(acts[l], (size_t)batch * sizes[l + 1] * sizeof(float), "acts[l]");
  }
  size_t need = 0;
  for (int l = 0; l < layers; ++l) need = std::max(need, gemm_ws_floats(batch, sizes[l + 1], sizes[l]));
  st = ensure_ws(h, need * sizeof(float) + 256);
  if (st) return st;
  float* part = (float*)h->ws;
  hipStream_t s = (hipStream_t)stream;
  const bool bf = compute == RTR_BF16;
  for (int l = 0; l < layers; ++l) {
    const float* in = l == 0 ? x : acts[l - 1];
    float* out = l == layers - 1 ? y : acts[l];
    st = run_gemm(h, bf, in, sizes[l], 1, W[l], sizes[l + 1], 1, batch, sizes[l + 1], sizes[l],
                  part, b[l], nullptr, l < layers - 1 ? 1 : 0, out, s);
    if (st) return st;
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_core_loss(rtr_handle h, const float* y, const float* target, int32_t batch,
                             int64_t per_row, float grad_scale, float* loss, float* dy,
                             void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (batch < 1 || per_row < 1 || per_row > (1 << 30))
    return fail(h, RTR_ERR_INVALID_ARG, "need batch >= 1 and 1 <= per_row <= 2^30");
  CHECK_DEV(y, (size_t)batch * per_row * sizeof(float), "y");
  CHECK_DEV(target, (size_t)batch * per_row * sizeof(float), "target");
  CHECK_DEV(dy, (size_t)batch * per_row * sizeof(float), "dy");
  CHECK_DEV(loss, (size_t)batch * sizeof(float), "loss");
  HIP_TRY(rtr::launch_core_loss(y, target, (int)per_row, grad_scale, batch, loss, dy,
                                (hipStream_t)stream),
          "core loss");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_tr_loss(rtr_handle h, const float* y, const float* target, int32_t batch,
                           const int32_t* K, const int32_t* R, float grad_scale, float* loss,
                           float* dy, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (!y || !target || !loss || !dy || !K || !R || batch < 1)
    return fail(h, RTR_ERR_INVALID_ARG, "bad arguments");
  rtr::TrLoss4 sh{};
  int dout = 0;
  for (int n = 0; n < 4; ++n) {
    if (K[n] < 1 || R[n] < 1 || R[n] > 8) return fail(h, RTR_ERR_INVALID_ARG, "need K_n >= 1, 1 <= R_n <= 8");
    sh.K[n] = K[n];
    sh.R[n] = R[n];
    dout += R[n] * K[n] * R[(n + 1) % 4];
  }
  sh.zpad = (dout + 63) & ~63;
  {
    const size_t pk = (size_t)K[0] * K[1] * K[2] * K[3];
    CHECK_DEV(y, (size_t)batch * dout * sizeof(float), "y");
    CHECK_DEV(dy, (size_t)batch * dout * sizeof(float), "dy");
    CHECK_DEV(target, (size_t)batch * pk * sizeof(float), "target");
    CHECK_DEV(loss, (size_t)batch * sizeof(float), "loss");
  }
  const size_t lds = rtr::tr_loss4_lds(sh);
  if (lds > 150 * 1024)
    return fail(h, RTR_ERR_UNSUPPORTED, "K_1 K_2 K_3 K_4 too large for the per-sample work-group");
  HIP_TRY(rtr::launch_tr_loss4(y, target, dout, sh, grad_scale, batch, loss, dy, (hipStream_t)stream),
          "tr loss");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_backward(rtr_handle h, int32_t layers, const int32_t* sizes,
                            const float* const* W, const float* x, int32_t batch,
                            const float* const* acts, const float* dy, float* const* dW,
                            float* const* db, rtr_dtype compute, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  st = check_mlp(h, layers, sizes, batch, compute);
  if (st) return st;
  if (!W || !x || !dy || !dW || !db || (layers > 1 && !acts))
    return fail(h, RTR_ERR_INVALID_ARG, "W, x, dy, dW, db (and acts for hidden layers) required");
  CHECK_DEV(x, (size_t)batch * sizes[0] * sizeof(float), "x");
  CHECK_DEV(dy, (size_t)batch * sizes[layers] * sizeof(float), "dy");
  for (int l = 0; l < layers; ++l) {
    CHECK_DEV(W[l], (size_t)sizes[l] * sizes[l + 1] * sizeof(float), "W[l]");
    CHECK_DEV(dW[l], (size_t)sizes[l] * sizes[l + 1] * sizeof(float), "dW[l]");
    CHECK_DEV(db[l], (size_t)sizes[l + 1] * sizeof(float), "db[l]");
    if (l < layers - 1) CHECK_DEV(acts[l], (size_t)batch * sizes[l + 1] * sizeof(float), "acts[l]");
  }
  size_t need = 0, gmax = 0;
  for (int l = 0; l < layers; ++l) {
    need = std::max(need, gemm_ws_floats(sizes[l], sizes[l + 1], batch));
    if (l > 0) need = std::max(need, gemm_ws_floats(batch, sizes[l], sizes[l + 1]));
    gmax = std::max(gmax, (size_t)batch * sizes[l]);
  }
  Carve plan(nullptr);
  plan.take<float>(need);
  plan.take<float>(gmax);
  plan.take<float>(gmax);
  st = ensure_ws(h, plan.off);
  if (st) return st;
  Carve c(h->ws);
  float* part = c.take<float>(need);
  float* gb[2] = {c.take<float>(gmax), c.take<float>(gmax)};
  hipStream_t s = (hipStream_t)stream;
  const bool bf = compute == RTR_BF16;
  const float* g = dy;
  for (int l = layers - 1; l >= 0; --l) {
    const float* in = l == 0 ? x : acts[l - 1];
    const int64_t ni = sizes[l], no = sizes[l + 1];
    // dW_l = in^T g   (ni x no, contraction over the batch)
    st = run_gemm(h, bf, in, 1, ni, g, no, 1, ni, no, batch, part, nullptr, nullptr, 0, dW[l], s);
    if (st) return st;
    HIP_TRY(rtr::launch_colsum(g, batch, no, db[l], s), "bias gradient");
    if (l > 0) {
      // g_{l-1} = (g W_l^T) * (acts[l-1] > 0)
      float* gn = gb[l & 1];
      st = run_gemm(h, bf, g, no, 1, W[l], 1, no, batch, ni, no, part, nullptr, acts[l - 1], 2, gn, s);
      if (st) return st;
      g = gn;
    }
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_adam(rtr_handle h, float* w, const float* g, float* m, float* v, int64_t n,
                        double lr, double beta1, double beta2, double eps, int32_t step,
                        void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (!w || !g || !m || !v || n < 1 || step < 1) return fail(h, RTR_ERR_INVALID_ARG, "bad arguments");
  CHECK_DEV(w, (size_t)n * sizeof(float), "w");
  CHECK_DEV(g, (size_t)n * sizeof(float), "g");
  CHECK_DEV(m, (size_t)n * sizeof(float), "m");
  CHECK_DEV(v, (size_t)n * sizeof(float), "v");
  HIP_TRY(rtr::launch_adam(w, g, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream), "adam");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_mlp_to_cores(rtr_handle h, const float* y, int64_t per_row, int32_t rows,
                            const double* p_norm2, int32_t order, double* Z, void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (!y || !Z || per_row < 1 || rows < 1 || order < 1) return fail(h, RTR_ERR_INVALID_ARG, "bad arguments");
  CHECK_DEV(y, (size_t)per_row * rows * sizeof(float), "y");
  CHECK_DEV(Z, (size_t)per_row * rows * sizeof(double), "Z");
  if ((st = check_dev_opt(h, p_norm2, (size_t)rows * sizeof(double), "p_norm2"))) return st;
  HIP_TRY(rtr::launch_to_f64(y, per_row * rows, per_row, p_norm2, order, Z, (hipStream_t)stream),
          "to f64");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_backproject(rtr_handle h, int32_t order, const int64_t* dims, const int32_t* K,
                           const int32_t* R, const double* Z, const double* Q, double* G,
                           void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, K))) return st;
  if (!K || !R) return fail(h, RTR_ERR_INVALID_ARG, "K and R must be host arrays");
  if (!Z || !Q || !G) return fail(h, RTR_ERR_INVALID_ARG, "Z, Q and G must be device pointers");
  for (int n = 0; n < order; ++n)
    if (R[n] < 1 || R[n] > RTR_MAX_RANK) return fail(h, RTR_ERR_INVALID_ARG, "rank out of range");
  {
    size_t zb = 0, gb = 0;
    for (int n = 0; n < order; ++n) {
      const size_t rr = (size_t)R[n] * R[(n + 1) % order];
      zb += rr * keff(dims, K, n);
      gb += rr * dims[n];
    }
    CHECK_DEV(Z, zb * sizeof(double), "Z");
    CHECK_DEV(Q, q_bytes(dims, K, order), "Q");
    CHECK_DEV(G, gb * sizeof(double), "G");
  }
  hipStream_t s = (hipStream_t)stream;
  size_t zo = 0, qo = 0, go = 0;
  for (int n = 0; n < order; ++n) {
    const int Ra = R[n], Rb = R[(n + 1) % order];
    const int64_t k = keff(dims, K, n);
    HIP_TRY(rtr::launch_backproject(Z + zo, Q + qo, Ra, (int)k, dims[n], Rb, G + go, s),
            "backproject");
    zo += (size_t)Ra * k * Rb;
    qo += (size_t)dims[n] * k;
    go += (size_t)Ra * dims[n] * Rb;
  }
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_residual(rtr_handle h, const void* X, rtr_dtype x_dtype, int32_t order,
                        const int64_t* dims, const int32_t* R, const double* G, double* out,
                        void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if ((st = check_shape(h, order, dims, nullptr))) return st;
  if (order < 2) return fail(h, RTR_ERR_INVALID_ARG, "residual needs order >= 2");
  if (!R) return fail(h, RTR_ERR_INVALID_ARG, "R is NULL");
  if (!X || !G || !out) return fail(h, RTR_ERR_INVALID_ARG, "X, G and out must be device pointers");
  if (x_dtype != RTR_F64 && x_dtype != RTR_F32)
    return fail(h, RTR_ERR_UNSUPPORTED, "X must be FP64 or FP32");
  for (int n = 0; n < order; ++n)
    if (R[n] < 1 || R[n] > RTR_MAX_RANK) return fail(h, RTR_ERR_INVALID_ARG, "rank out of range");
  {
    size_t gb = 0;
    for (int n = 0; n < order; ++n) gb += (size_t)R[n] * dims[n] * R[(n + 1) % order];
    CHECK_DEV(X, x_bytes(dims, order, x_dtype), "X");
    CHECK_DEV(G, gb * sizeof(double), "G");
    CHECK_DEV(out, 2 * sizeof(double), "out");
  }
  hipStream_t s = (hipStream_t)stream;
  const int hm = order / 2;
  int64_t IL = 1, IR = 1;
  for (int n = 0; n < hm; ++n) IL *= dims[n];
  for (int n = hm; n < order; ++n) IR *= dims[n];
  const int RR = R[0] * R[hm];
  const bool f32 = x_dtype == RTR_F32;
  const int64_t nblocks = rtr::residual_blocks(f32, IL, IR, RR);
  const int RRp = (RR + 3) & ~3;
  Carve plan(nullptr);
  plan.take<double>((size_t)IL * RR);
  plan.take<double>((size_t)IR * RR);
  plan.take<double>((size_t)2 * nblocks);
  plan.take<float>(f32 ? (size_t)(IL + IR) * RRp : 1);
  if ((st = ensure_ws(h, plan.off + 256))) return st;
  Carve cv(h->ws);
  double* L = cv.take<double>((size_t)IL * RR);
  double* RtT = cv.take<double>((size_t)IR * RR);
  double* partial = cv.take<double>((size_t)2 * nblocks);
  float* lr32 = cv.take<float>(f32 ? (size_t)(IL + IR) * RRp : 1);
  size_t goff[RTR_MAX_ORDER];
  size_t go = 0;
  for (int n = 0; n < order; ++n) {
    goff[n] = go;
    go += (size_t)R[n] * dims[n] * R[(n + 1) % order];
  }
  rtr::Chain cl{}, cr{};
  cl.L = hm;
  for (int n = 0; n < hm; ++n) {
    cl.core[n] = G + goff[n];
    cl.I[n] = (int)dims[n];
    cl.Ra[n] = R[n];
    cl.Rb[n] = R[(n + 1) % order];
  }
  cr.L = order - hm;
  for (int n = hm; n < order; ++n) {
    cr.core[n - hm] = G + goff[n];
    cr.I[n - hm] = (int)dims[n];
    cr.Ra[n - hm] = R[n];
    cr.Rb[n - hm] = R[(n + 1) % order];
  }
  HIP_TRY(rtr::launch_chain(cl, IL, 0, L, nullptr, s), "chain");
  HIP_TRY(rtr::launch_chain(cr, IR, 1, RtT, nullptr, s), "chain");
  HIP_TRY(rtr::launch_residual(f32, X, IL, IR, RR, L, RtT, partial, lr32, out, s), "residual");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_normals(rtr_handle h, uint64_t seed, uint32_t stream_word, uint32_t tensor_id,
                       int64_t start, int64_t count, rtr_dtype dtype, void* out,
                       void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (start < 0 || count < 0) return fail(h, RTR_ERR_INVALID_ARG, "start and count must be >= 0");
  if (count > 0 && !out) return fail(h, RTR_ERR_INVALID_ARG, "out must be a device pointer");
  if (dtype != RTR_F64 && dtype != RTR_F32)
    return fail(h, RTR_ERR_UNSUPPORTED, "normals are FP64 or FP32");
  if (count > 0) CHECK_DEV(out, (size_t)count * (dtype == RTR_F64 ? 8 : 4), "out");
  HIP_TRY(rtr::launch_normals(dtype == RTR_F32, seed, stream_word, tensor_id, start, count, out,
                              (hipStream_t)stream),
          "normals");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_read_probe(rtr_handle h, const void* x, int64_t bytes, double* out,
                          void* stream) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  Guard guard(h);
  if (bytes < 16 || bytes % 16 != 0 || ((uintptr_t)x & 15) != 0)
    return fail(h, RTR_ERR_INVALID_ARG, "x must be 16-byte aligned and bytes a positive multiple of 16");
  CHECK_DEV(x, (size_t)bytes, "x");
  CHECK_DEV(out, sizeof(double), "out");
  const int blocks = rtr::probe_blocks();
  if ((st = ensure_ws(h, (size_t)blocks * sizeof(double) + 256))) return st;
  HIP_TRY(rtr::launch_read_probe(x, bytes, (double*)h->ws, out, (hipStream_t)stream), "read probe");
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

// ---------------------------------------------------------------------------------------
rtr_status rtr_status_sync(rtr_handle h, void* stream, uint32_t* bits) try {
  rtr_status st = check_handle(h);
  if (st) return st;
  unsigned v = 0;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(&v, h->status, sizeof(unsigned), hipMemcpyDeviceToHost), "hipMemcpy");
  HIP_TRY(hipMemset(h->status, 0, sizeof(unsigned)), "hipMemset");
  if (bits) *bits = v;
  return v ? fail(h, RTR_ERR_NUMERICAL, "device status bits set") : RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

rtr_status rtr_batch_set_work_lists(rtr_handle h, int32_t on) {
  if (!h || on < 0 || on > 1) return RTR_ERR_INVALID_ARG;
  h->bt_lists = on;
  return RTR_OK;
}

rtr_status rtr_set_als_launch(rtr_handle h, int32_t mode) {
  if (!h || mode < 0 || mode > 1) return RTR_ERR_INVALID_ARG;
  h->als_launch = mode;
  return RTR_OK;
}

rtr_status rtr_profile_enable(rtr_handle h, int32_t on) {
  if (!h) return RTR_ERR_INVALID_ARG;
  if (on < 0 || on > 2) return RTR_ERR_INVALID_ARG;
  h->prof_level = on;
  return RTR_OK;
}

rtr_status rtr_profile_reset(rtr_handle h) {
  if (!h) return RTR_ERR_INVALID_ARG;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (auto& r : h->recs) {
    h->pool.push_back(r.e0);
    h->pool.push_back(r.e1);
  }
  h->recs.clear();
  return RTR_OK;
}

rtr_status rtr_profile_read(rtr_handle h, const char* name, double* total_ms, int64_t* launches) try {
  if (!h || !name) return RTR_ERR_INVALID_ARG;
  HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
  HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : h->recs) {
    if (std::strcmp(r.name, name) != 0) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.e0, r.e1), "hipEventElapsedTime");
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return RTR_OK;
} catch (...) {
  return fail(h, RTR_ERR_INTERNAL, "unexpected exception");
}

}  // extern "C"
