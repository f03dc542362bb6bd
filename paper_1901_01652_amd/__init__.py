"""Python binding of librtr.so, the gfx950 randomized tensor-ring decomposition library.

Argument marshalling only: every stage runs in the library's HIP kernels.  torch tensors
supply device memory and the current HIP stream.  Importing this package fails loudly if
librtr.so has not been built (``python paper_1901_01652_amd/build.py``); there is no CPU
fallback.

The functions mirror the C ABI of include/rtr.h (Yuan et al., arXiv:1901.01652, Alg. 1):
  rtr_sketch       steps 3-6 (+ power iterations)  -> packed Q_n
  rtr_compress     step 7, Eq. (3)                  -> P
  rtr_decompose    step 9 (TR-ALS)                  -> packed cores Z_n, error trace
  rtr_backproject  steps 10-12                      -> packed cores G_n
  rtr_residual     Sec. 4 error measure             -> [||X - Psi(G)||^2, ||X||^2]
"""
import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rtr.h")

RTR_F64, RTR_F32, RTR_BF16, RTR_FP8_E4M3 = 0, 1, 2, 3
RTR_METHOD_ALS, RTR_METHOD_SVD = 0, 1
RTR_OK, RTR_ERR_INVALID_ARG, RTR_ERR_UNSUPPORTED = 0, 1, 2
RTR_STATUS_CHOLESKY_FAILED = 0x1
RTR_STATUS_RANK_CAPPED = 0x2
RTR_STATUS_SYNC_TIMEOUT = 0x4
RTR_STATUS_INDEX_RANGE = 0x8
MAX_ORDER = 8

_DTYPES = {"f64": RTR_F64, "f32": RTR_F32, "bf16": RTR_BF16, "fp8": RTR_FP8_E4M3}


class RtrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("max_sweeps", ctypes.c_int32),
                ("tol", ctypes.c_double), ("eps", ctypes.c_double)]


class _AlsItem(ctypes.Structure):
    _fields_ = [("P", ctypes.c_void_p), ("Z_init", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("err_trace", ctypes.c_void_p), ("sweeps_run", ctypes.c_void_p),
                ("order", ctypes.c_int32), ("Kp", ctypes.c_int32 * 8), ("R", ctypes.c_int32 * 8)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("order", ctypes.c_int32), ("dims", ctypes.c_int64 * 8),
                ("K", ctypes.c_int32 * 8), ("R", ctypes.c_int32 * 8), ("seed", ctypes.c_uint64),
                ("tensor_id", ctypes.c_uint32), ("Z_init", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("G", ctypes.c_void_p),
                ("err_trace", ctypes.c_void_p), ("sweeps_run", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python paper_1901_01652_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.c_double)
    P64 = ctypes.POINTER(i64)
    P32 = ctypes.POINTER(i32)
    sig = {
        "rtr_create": [ctypes.c_int, ctypes.POINTER(vp)],
        "rtr_destroy": [vp],
        "rtr_sketch": [vp, vp, ctypes.c_int, i32, P64, P32, i32, u64, u32, ctypes.c_int, vp, vp],
        "rtr_sketch_noalloc": [vp, vp, ctypes.c_int, i32, P64, P32, i32, u64, u32, ctypes.c_int, vp,
                               vp],
        "rtr_sketch_kr": [vp, vp, ctypes.c_int, i32, P64, P32, i32, u64, u32, ctypes.c_int, vp, vp,
                          vp],
        "rtr_sketch_sequential": [vp, vp, ctypes.c_int, i32, P64, P32, u64, u32, ctypes.c_int, vp,
                                  vp, vp, vp],
        "rtr_sketch_coo": [vp, vp, vp, ctypes.c_int, i64, i32, P64, P32, u64, u32, vp, vp, vp],
        "rtr_compress_coo": [vp, vp, vp, ctypes.c_int, i64, i32, P64, P32, vp, vp, vp, vp],
        "rtr_compress": [vp, vp, ctypes.c_int, i32, P64, P32, vp, ctypes.c_int, vp, vp, vp],
        "rtr_decompose": [vp, vp, i32, P32, P32, ctypes.POINTER(_Opts), vp, vp, vp, vp, vp],
        "rtr_decompose_svd": [vp, vp, i32, P32, P32, dp, vp, vp, vp, vp],
        "rtr_decompose_batch": [vp, ctypes.POINTER(_AlsItem), i32, i32, dp, vp],
        "rtr_batch_run": [vp, ctypes.POINTER(_BatchItem), i32, ctypes.c_int, ctypes.c_int, i32, i32,
                          dp, i32, vp],
        "rtr_batch_autotune": [vp, ctypes.POINTER(_BatchItem), i32, ctypes.c_int, ctypes.c_int, P32, vp],
        "rtr_backproject": [vp, i32, P64, P32, P32, vp, vp, vp, vp],
        "rtr_mlp_normalize": [vp, vp, i64, i32, vp, vp],
        "rtr_mlp_forward": [vp, i32, P32, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, i32,
                            ctypes.POINTER(vp), vp, ctypes.c_int, vp],
        "rtr_mlp_tr_loss": [vp, vp, vp, i32, P32, P32, ctypes.c_float, vp, vp, vp],
        "rtr_mlp_core_loss": [vp, vp, vp, i32, i64, ctypes.c_float, vp, vp, vp],
        "rtr_mlp_backward": [vp, i32, P32, ctypes.POINTER(vp), vp, i32, ctypes.POINTER(vp), vp,
                             ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, vp],
        "rtr_mlp_adam": [vp, vp, vp, vp, vp, i64, dp, dp, dp, dp, i32, vp],
        "rtr_mlp_to_cores": [vp, vp, i64, i32, vp, i32, vp, vp],
        "rtr_residual": [vp, vp, ctypes.c_int, i32, P64, P32, vp, vp, vp],
        "rtr_normals": [vp, u64, u32, u32, i64, i64, ctypes.c_int, vp, vp],
        "rtr_status_sync": [vp, vp, ctypes.POINTER(u32)],
        "rtr_profile_enable": [vp, i32],
        "rtr_read_probe": [vp, vp, i64, vp, vp],
        "rtr_set_als_launch": [vp, i32],
        "rtr_batch_set_work_lists": [vp, i32],
        "rtr_profile_reset": [vp],
        "rtr_profile_read": [vp, ctypes.c_char_p, ctypes.POINTER(dp), P64],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.rtr_last_error.argtypes = [vp]
    lib.rtr_last_error.restype = ctypes.c_char_p
    lib.rtr_status_string.argtypes = [ctypes.c_int]
    lib.rtr_status_string.restype = ctypes.c_char_p
    return lib


lib = _load()


def header_symbols():
    """Function names declared in include/rtr.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rtr_status|const char\*)\s+(rtr_\w+)\s*\(", txt, re.M)))


def status_string(code):
    return lib.rtr_status_string(int(code)).decode()


class Handle:
    """Owns an rtr_handle (device workspace, status word, timing records)."""

    def __init__(self, device=0):
        self.ptr = ctypes.c_void_p()
        st = lib.rtr_create(int(device), ctypes.byref(self.ptr))
        if st != 0:
            raise RtrError(st, f"rtr_create({device}) failed: {status_string(st)}")
        self.device = device

    def close(self):
        if self.ptr:
            lib.rtr_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib.rtr_last_error(self.ptr).decode()

    def check(self, st):
        if st != 0:
            raise RtrError(st, f"{status_string(st)}: {self.last_error()}")


def _i64(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def _i32(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()


def _stream(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _xdtype(X):
    if X.dtype == torch.float64:
        return RTR_F64
    if X.dtype == torch.float32:
        return RTR_F32
    raise TypeError("X must be float64 or float32")


def keff(dims, K):
    return [min(int(k), int(d)) for k, d in zip(K, dims)]


def q_size(dims, K):
    return sum(d * k for d, k in zip(dims, keff(dims, K)))


def core_shapes(D, R):
    N = len(D)
    return [(int(R[n]), int(D[n]), int(R[(n + 1) % N])) for n in range(N)]


def pack(cores, device=None, dtype=torch.float64):
    """Concatenate cores (or Q_n) into one flat tensor in the packed layout."""
    parts = [torch.as_tensor(c, dtype=dtype).reshape(-1) for c in cores]
    out = torch.cat(parts)
    return out.to(device) if device is not None else out


def unpack(flat, shapes):
    """Views of a packed buffer as tensors of the given shapes."""
    out, off = [], 0
    for s in shapes:
        n = 1
        for x in s:
            n *= x
        out.append(flat[off:off + n].view(*s))
        off += n
    return out


def q_shapes(dims, K):
    return [(int(d), k) for d, k in zip(dims, keff(dims, K))]


def rtr_sketch(h, X, K, power_iters=0, seed=0, tensor_id=0, compute=None, Q=None, stream=None,
               projection="gaussian", x_norm2=None):
    """Alg. 1 steps 3-6: packed FP64 Q_n (I_n x K'_n) of tensor X (device).  ``projection``
    "khatri_rao" calls rtr_sketch_kr (structured test matrices; ``x_norm2``, a device FP64
    scalar, then receives ||X||^2)."""
    dims = list(X.shape)
    assert X.is_contiguous()
    xd = _xdtype(X)
    cd = xd if compute is None else _DTYPES[compute]
    if Q is None:
        Q = torch.empty(q_size(dims, K), dtype=torch.float64, device=X.device)
    args = [h.ptr, _ptr(X), xd, len(dims), _i64(dims), _i32(K), int(power_iters), int(seed),
            int(tensor_id), cd, _ptr(Q)]
    if projection == "khatri_rao":
        h.check(lib.rtr_sketch_kr(*args, _ptr(x_norm2) if x_norm2 is not None else None,
                                  _stream(stream, X.device)))
    elif projection == "gaussian":
        assert x_norm2 is None, "||X||^2 comes with the Khatri-Rao sketch"
        h.check(lib.rtr_sketch(*args, _stream(stream, X.device)))
    else:
        raise ValueError(projection)
    return Q


def rtr_sketch_sequential(h, X, K, seed=0, tensor_id=0, compute=None, Q=None, P=None,
                          p_norm2=None, stream=None):
    """Alg. 1 steps 3-8 with step 7 read sequentially: returns (packed Q_n, P)."""
    dims = list(X.shape)
    assert X.is_contiguous()
    xd = _xdtype(X)
    cd = xd if compute is None else _DTYPES[compute]
    if Q is None:
        Q = torch.empty(q_size(dims, K), dtype=torch.float64, device=X.device)
    if P is None:
        P = torch.empty(keff(dims, K), dtype=torch.float64, device=X.device)
    h.check(lib.rtr_sketch_sequential(h.ptr, _ptr(X), xd, len(dims), _i64(dims), _i32(K), int(seed),
                                      int(tensor_id), cd, _ptr(Q), _ptr(P),
                                      _ptr(p_norm2) if p_norm2 is not None else None,
                                      _stream(stream, X.device)))
    return Q, P


def _coo(indices, values):
    assert indices.dtype == torch.int64 and indices.dim() == 2 and indices.is_contiguous()
    assert values.dim() == 1 and values.is_contiguous() and values.shape[0] == indices.shape[0]
    return _xdtype(values), int(indices.shape[0])


def rtr_sketch_coo(h, indices, values, dims, K, seed=0, tensor_id=0, Q=None, x_norm2=None,
                   stream=None):
    """Alg. 1 steps 3-6 for a tensor given by its nonzeros (``indices`` nnz x N int64,
    ``values`` nnz FP64/FP32, both on the device): packed FP64 Q_n."""
    vd, nnz = _coo(indices, values)
    if Q is None:
        Q = torch.empty(q_size(dims, K), dtype=torch.float64, device=values.device)
    h.check(lib.rtr_sketch_coo(h.ptr, _ptr(indices), _ptr(values), vd, nnz, len(dims), _i64(dims),
                               _i32(K), int(seed), int(tensor_id), _ptr(Q), _ptr(x_norm2),
                               _stream(stream, values.device)))
    return Q


def rtr_compress_coo(h, indices, values, dims, K, Q, P=None, p_norm2=None, stream=None):
    """Alg. 1 step 7 / Eq. (3) for a tensor given by its nonzeros: P (K'_1 x .. x K'_N, FP64)."""
    vd, nnz = _coo(indices, values)
    if P is None:
        P = torch.empty(keff(dims, K), dtype=torch.float64, device=values.device)
    h.check(lib.rtr_compress_coo(h.ptr, _ptr(indices), _ptr(values), vd, nnz, len(dims),
                                 _i64(dims), _i32(K), _ptr(Q), _ptr(P), _ptr(p_norm2),
                                 _stream(stream, values.device)))
    return P


def rtr_sketch_noalloc(h, X, K, Q, power_iters=0, seed=0, tensor_id=0, compute=None, stream=None):
    """rtr_sketch without device allocation (fixed per-GPU scratch); ``Q`` is caller-owned."""
    dims = list(X.shape)
    assert X.is_contiguous()
    xd = _xdtype(X)
    cd = xd if compute is None else _DTYPES[compute]
    h.check(lib.rtr_sketch_noalloc(h.ptr, _ptr(X), xd, len(dims), _i64(dims), _i32(K),
                                   int(power_iters), int(seed), int(tensor_id), cd, _ptr(Q),
                                   _stream(stream, X.device)))
    return Q


def rtr_compress(h, X, K, Q, compute=None, P=None, p_norm2=None, stream=None):
    """Alg. 1 step 7 / Eq. (3): P (K'_1 x .. x K'_N, FP64) from X and packed Q."""
    dims = list(X.shape)
    assert X.is_contiguous()
    xd = _xdtype(X)
    cd = xd if compute is None else _DTYPES[compute]
    if P is None:
        P = torch.empty(keff(dims, K), dtype=torch.float64, device=X.device)
    h.check(lib.rtr_compress(h.ptr, _ptr(X), xd, len(dims), _i64(dims), _i32(K), _ptr(Q), cd,
                             _ptr(P), _ptr(p_norm2), _stream(stream, X.device)))
    return P


def rtr_decompose(h, P, R, Z_init, max_sweeps, tol=0.0, method="als", eps=0.0, Z=None,
                  err_trace=None, sweeps_run=None, stream=None):
    """Alg. 1 step 9: TR-ALS on P from packed Z_init; returns (Z, err_trace, sweeps_run)."""
    Kp = list(P.shape)
    if Z is None:
        Z = torch.empty_like(Z_init)
    if err_trace is None:
        err_trace = torch.zeros(max_sweeps, dtype=torch.float64, device=P.device)
    if sweeps_run is None:
        sweeps_run = torch.zeros(1, dtype=torch.int32, device=P.device)
    opts = _Opts(RTR_METHOD_ALS if method == "als" else RTR_METHOD_SVD, int(max_sweeps), float(tol),
                 float(eps))
    h.check(lib.rtr_decompose(h.ptr, _ptr(P), len(Kp), _i32(Kp), _i32(R), ctypes.byref(opts),
                              _ptr(Z_init), _ptr(Z), _ptr(err_trace), _ptr(sweeps_run),
                              _stream(stream, P.device)))
    return Z, err_trace, sweeps_run


def svd_slots(Kp, Rcap):
    """Slot sizes (doubles) of the TR-SVD core buffer: Rcap_n * K'_n * Rcap_{n+1}."""
    N = len(Kp)
    return [int(Rcap[n]) * int(Kp[n]) * int(Rcap[(n + 1) % N]) for n in range(N)]


def rtr_decompose_svd(h, P, Rcap, eps, Z=None, ranks=None, err=None, stream=None):
    """Alg. 1 step 9 with TR-SVD.  Returns the device outputs (Z slots, ranks, err); use
    ``svd_cores`` to read the cores out."""
    Kp = list(P.shape)
    if Z is None:
        Z = torch.zeros(sum(svd_slots(Kp, Rcap)), dtype=torch.float64, device=P.device)
    if ranks is None:
        ranks = torch.zeros(len(Kp), dtype=torch.int32, device=P.device)
    if err is None:
        err = torch.zeros(1, dtype=torch.float64, device=P.device)
    h.check(lib.rtr_decompose_svd(h.ptr, _ptr(P), len(Kp), _i32(Kp), _i32(Rcap), float(eps),
                                  _ptr(Z), _ptr(ranks), _ptr(err), _stream(stream, P.device)))
    return Z, ranks, err


def svd_cores(Z, ranks, Kp, Rcap):
    """The cores (R_n, K'_n, R_{n+1}) stored at the start of each TR-SVD slot."""
    N = len(Kp)
    R = [int(r) for r in ranks]
    out, off = [], 0
    for n, size in enumerate(svd_slots(Kp, Rcap)):
        shape = (R[n], int(Kp[n]), R[(n + 1) % N])
        cnt = shape[0] * shape[1] * shape[2]
        out.append(Z[off:off + cnt].view(*shape))
        off += size
    return out


def _arr8(ctype, vals):
    a = (ctype * 8)()
    for i, v in enumerate(vals):
        a[i] = int(v)
    return a


def rtr_decompose_batch(h, items, max_sweeps, tol=0.0, stream=None):
    """Batched TR-ALS in one launch.  ``items``: dicts with P (device FP64 tensor), R, Z_init
    (packed, device); optional Z, err_trace, sweeps_run.  Fills and returns the dicts."""
    arr = (_AlsItem * len(items))()
    for t, it in enumerate(items):
        P = it["P"]
        dev = P.device
        it.setdefault("Z", torch.empty_like(it["Z_init"]))
        it.setdefault("err_trace", torch.zeros(max_sweeps, dtype=torch.float64, device=dev))
        it.setdefault("sweeps_run", torch.zeros(1, dtype=torch.int32, device=dev))
        a = arr[t]
        a.P, a.Z_init, a.Z = P.data_ptr(), it["Z_init"].data_ptr(), it["Z"].data_ptr()
        a.err_trace, a.sweeps_run = it["err_trace"].data_ptr(), it["sweeps_run"].data_ptr()
        a.order = P.dim()
        a.Kp = _arr8(ctypes.c_int32, P.shape)
        a.R = _arr8(ctypes.c_int32, it["R"])
    dev = items[0]["P"].device
    h.check(lib.rtr_decompose_batch(h.ptr, arr, len(items), int(max_sweeps), float(tol),
                                    _stream(stream, dev)))
    return items


def _batch_items(items, max_sweeps):
    arr = (_BatchItem * len(items))()
    xdt = _xdtype(items[0]["X"])
    for t, it in enumerate(items):
        X = it["X"]
        dev = X.device
        dims = list(X.shape)
        K, R = list(it["K"]), list(it["R"])
        Kp = [min(k, d) for k, d in zip(K, dims)]
        f64 = dict(dtype=torch.float64, device=dev)
        it.setdefault("Q", torch.empty(sum(d * k for d, k in zip(dims, Kp)), **f64))
        it.setdefault("P", torch.empty(Kp, **f64))
        it.setdefault("Z", torch.empty_like(it["Z_init"]))
        it.setdefault("G", torch.empty(sum(a * b * c for a, b, c in core_shapes(dims, R)), **f64))
        it.setdefault("err_trace", torch.zeros(max_sweeps, **f64))
        it.setdefault("sweeps_run", torch.zeros(1, dtype=torch.int32, device=dev))
        a = arr[t]
        a.X, a.order = X.data_ptr(), len(dims)
        a.dims, a.K, a.R = _arr8(ctypes.c_int64, dims), _arr8(ctypes.c_int32, K), _arr8(ctypes.c_int32, R)
        a.seed, a.tensor_id = int(it.get("seed", 0)), int(it.get("tensor_id", 0))
        a.Z_init = it["Z_init"].data_ptr()
        for name in ("Q", "P", "Z", "G", "err_trace", "sweeps_run"):
            setattr(a, name, it[name].data_ptr() if it[name] is not None else None)
    return arr, xdt


def rtr_batch_run(h, items, max_sweeps, compute=None, power_iters=0, tol=0.0, use_graph=False,
                  stream=None):
    """Alg. 1 steps 3-12 for a batch.  ``items``: dicts with X (device), K, R, Z_init (packed,
    device), seed, tensor_id; outputs Q, P, Z, G, err_trace, sweeps_run are allocated when
    missing (keep the dicts to replay the same batch as a graph)."""
    arr, xdt = _batch_items(items, max_sweeps)
    if compute is None:
        compute = "f64" if xdt == RTR_F64 else "f32"
    dev = items[0]["X"].device
    h.check(lib.rtr_batch_run(h.ptr, arr, len(items), xdt, _DTYPES[compute], int(power_iters),
                              int(max_sweeps), float(tol), int(bool(use_graph)), _stream(stream, dev)))
    return items


def rtr_batch_autotune(h, items, compute="f32", table_path=None, stream=None):
    """Times the batched work lists' tile candidates on ``items`` and keeps the fastest in the
    handle; returns the table (and writes it as JSON to ``table_path`` when given)."""
    arr, xdt = _batch_items(items, 1)
    tab = (ctypes.c_int32 * 8)()
    dev = items[0]["X"].device
    h.check(lib.rtr_batch_autotune(h.ptr, arr, len(items), xdt, _DTYPES[compute], tab,
                                   _stream(stream, dev)))
    table = {"sketch_chunks_per_job": tab[0], "ttm_outputs_per_thread": tab[1],
             "sketch_us": {"16": tab[2], "64": tab[3], "256": tab[4]},
             "ttm_us": {"4": tab[5], "16": tab[6], "64": tab[7]}}
    if table_path:
        import json
        with open(table_path, "w") as f:
            json.dump(table, f, indent=1)
    return table


def _ptrs(ts):
    return (ctypes.c_void_p * max(1, len(ts)))(*[t.data_ptr() for t in ts])


def rtr_mlp_normalize(h, P, out=None, stream=None):
    """Rows of P (batch x d, FP64) divided by their norms, FP32."""
    rows, d = P.shape[0], P[0].numel()
    if out is None:
        out = torch.empty((rows, d), dtype=torch.float32, device=P.device)
    h.check(lib.rtr_mlp_normalize(h.ptr, _ptr(P), d, rows, _ptr(out), _stream(stream, P.device)))
    return out


def rtr_mlp_forward(h, W, b, x, acts=None, y=None, compute="bf16", stream=None):
    """Forward pass; returns (y, acts)."""
    sizes = [W[0].shape[0]] + [w.shape[1] for w in W]
    B = x.shape[0]
    if acts is None:
        acts = [torch.empty((B, n), dtype=torch.float32, device=x.device) for n in sizes[1:-1]]
    if y is None:
        y = torch.empty((B, sizes[-1]), dtype=torch.float32, device=x.device)
    h.check(lib.rtr_mlp_forward(h.ptr, len(W), _i32(sizes), _ptrs(W), _ptrs(b), _ptr(x), B,
                                _ptrs(acts), _ptr(y), _DTYPES[compute], _stream(stream, x.device)))
    return y, acts


def rtr_mlp_core_loss(h, y, target, grad_scale, loss=None, dy=None, stream=None):
    """Supervised loss ||y - target||^2 per sample and its gradient (times grad_scale)."""
    B, d = y.shape
    if loss is None:
        loss = torch.empty(B, dtype=torch.float32, device=y.device)
    if dy is None:
        dy = torch.empty_like(y)
    h.check(lib.rtr_mlp_core_loss(h.ptr, _ptr(y), _ptr(target), B, d, float(grad_scale), _ptr(loss),
                                  _ptr(dy), _stream(stream, y.device)))
    return loss, dy


def rtr_mlp_tr_loss(h, y, target, K, R, grad_scale, loss=None, dy=None, stream=None):
    B = y.shape[0]
    if loss is None:
        loss = torch.empty(B, dtype=torch.float32, device=y.device)
    if dy is None:
        dy = torch.empty_like(y)
    h.check(lib.rtr_mlp_tr_loss(h.ptr, _ptr(y), _ptr(target), B, _i32(K), _i32(R),
                                float(grad_scale), _ptr(loss), _ptr(dy), _stream(stream, y.device)))
    return loss, dy


def rtr_mlp_backward(h, W, x, acts, dy, dW=None, db=None, compute="bf16", stream=None):
    sizes = [W[0].shape[0]] + [w.shape[1] for w in W]
    if dW is None:
        dW = [torch.empty_like(w) for w in W]
    if db is None:
        db = [torch.empty(w.shape[1], dtype=torch.float32, device=x.device) for w in W]
    h.check(lib.rtr_mlp_backward(h.ptr, len(W), _i32(sizes), _ptrs(W), _ptr(x), x.shape[0],
                                 _ptrs(acts), _ptr(dy), _ptrs(dW), _ptrs(db), _DTYPES[compute],
                                 _stream(stream, x.device)))
    return dW, db


def rtr_mlp_adam(h, w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    h.check(lib.rtr_mlp_adam(h.ptr, _ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), float(lr),
                             float(beta1), float(beta2), float(eps), int(step),
                             _stream(stream, w.device)))


def rtr_mlp_to_cores(h, y, p_norm2=None, order=4, Z=None, stream=None):
    """FP64 cores from predictions y (rows x per_row), each row scaled by ||P||^(1/order)."""
    y2 = y.reshape(-1, y.shape[-1])
    if Z is None:
        Z = torch.empty(y2.shape, dtype=torch.float64, device=y.device)
    h.check(lib.rtr_mlp_to_cores(h.ptr, _ptr(y2), y2.shape[1], y2.shape[0], _ptr(p_norm2),
                                 int(order), _ptr(Z), _stream(stream, y.device)))
    return Z


def rtr_backproject(h, dims, K, R, Z, Q, G=None, stream=None):
    """Alg. 1 steps 10-12: packed G_n = Z_n x_2 Q_n."""
    if G is None:
        G = torch.empty(sum(a * b * c for a, b, c in core_shapes(dims, R)), dtype=torch.float64,
                        device=Z.device)
    h.check(lib.rtr_backproject(h.ptr, len(dims), _i64(dims), _i32(K), _i32(R), _ptr(Z), _ptr(Q),
                                _ptr(G), _stream(stream, Z.device)))
    return G


def rtr_residual(h, X, R, G, out=None, stream=None):
    """Sec. 4: [||X - Psi(G)||^2, ||X||^2] (FP64, device)."""
    dims = list(X.shape)
    if out is None:
        out = torch.zeros(2, dtype=torch.float64, device=X.device)
    h.check(lib.rtr_residual(h.ptr, _ptr(X), _xdtype(X), len(dims), _i64(dims), _i32(R), _ptr(G),
                             _ptr(out), _stream(stream, X.device)))
    return out


def rtr_normals(h, seed, stream_word, tensor_id, start, count, dtype="f64", device=0, out=None,
                stream=None):
    """Elements [start, start+count) of the Gaussian stream of Alg. 1 step 4 (device tensor)."""
    td = torch.float64 if dtype == "f64" else torch.float32
    if out is None:
        out = torch.empty(int(count), dtype=td, device=f"cuda:{device}")
    h.check(lib.rtr_normals(h.ptr, int(seed), int(stream_word), int(tensor_id), int(start),
                            int(count), _DTYPES[dtype], _ptr(out), _stream(stream, out.device)))
    return out


def rtr_status_sync(h, stream=None, device=0):
    bits = ctypes.c_uint32(0)
    st = lib.rtr_status_sync(h.ptr, _stream(stream, device), ctypes.byref(bits))
    if st not in (0, 5):
        h.check(st)
    return int(bits.value)


def rtr_batch_set_work_lists(h, on):
    """1: rtr_batch_run takes the work lists where the batch allows (default); 0: per tensor."""
    h.check(lib.rtr_batch_set_work_lists(h.ptr, int(on)))


def rtr_set_als_launch(h, mode):
    """0: TR-ALS in one cooperative launch where supported (default); 1: two launches per update."""
    h.check(lib.rtr_set_als_launch(h.ptr, int(mode)))


def rtr_read_probe(h, x, out=None, stream=None):
    """HBM read-stream probe over the bytes of device tensor ``x`` (timed as "read_probe")."""
    if out is None:
        out = torch.zeros(1, dtype=torch.float64, device=x.device)
    h.check(lib.rtr_read_probe(h.ptr, _ptr(x), int(x.numel() * x.element_size()), _ptr(out),
                               _stream(stream, x.device)))
    return out


def rtr_profile_enable(h, level=1):
    """0 off, 1 kernels that stream X, 2 every kernel."""
    h.check(lib.rtr_profile_enable(h.ptr, int(level)))


def rtr_profile_reset(h):
    h.check(lib.rtr_profile_reset(h.ptr))


def rtr_profile_read(h, name):
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    h.check(lib.rtr_profile_read(h.ptr, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, int(n.value)
