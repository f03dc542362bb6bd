"""Seeded synthetic inputs for randomized tensor-ring decomposition.

Shared by the oracle-side tests and the GPU-side tests/benchmark; it holds none of the
decomposition's arithmetic (no sketch, QR, compression, ALS or back-projection).  It makes:

* TR cores with i.i.d. N(0,1) entries (Sec. 2.2 shapes R_n x I_n x R_{n+1}, R_{N+1} = R_1);
* the signal tensor S = Psi(cores) (element = trace of the product of core slices, Eq. 1),
  evaluated by merging the first half of the cores and the second half and contracting the
  two halves as one matrix product;
* i.i.d. Gaussian noise at a target SNR in dB: sigma^2 * numel = ||S||^2 10^(-SNR/10)
  (the noise levels of the paper's HSI experiment are quoted in dB);
* spatially smooth cores (Gaussian filter along the index, reflecting boundary) with the
  signal rescaled to [0, 1] for the hyperspectral-shaped workload;
* initial cores for TR-ALS (N(0,1)), which the decomposition takes as an input;
* the five workload definitions (small exact-arithmetic case, large dense sketch,
  hyperspectral-shaped, batched uneven, learned warm start).

Noise is keyed by the element's index in the FULL tensor: element e (row-major over the full
dims) is element e of a Philox4x32-10 Gaussian stream (Salmon et al., SC'11; Box-Muller on
word pairs, uniforms (w + 1/2) 2^-32), key (seed mod 2^32, seed >> 32), counter
(c mod 2^32, c >> 32, 0x03000000, tensor_id) with c = e >> 2 and lane e & 3.  A workload that
is the leading block of a larger one (``full_dims``) therefore gets exactly the noise of that
block of the larger tensor, and its noise level sigma is the larger tensor's (the signal norm
comes from the cores in closed form, ||Psi(G)||^2 = Tr prod_n sum_i G_n(i) (x) G_n(i)).
Signal and noise are formed in FP64 with torch on the requested device and rounded once to
the requested dtype.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

BASE_SEED = 20190105


def _rng(seed, tensor_id, tag):
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tensor_id), int(tag)]))


def tr_cores(seed, dims, ranks, tensor_id=0, tag=11):
    """Cores G_n (R_n, I_n, R_{n+1}) with N(0,1) entries, FP64 numpy."""
    rng = _rng(seed, tensor_id, tag)
    N = len(dims)
    return [rng.standard_normal((ranks[n], dims[n], ranks[(n + 1) % N])) for n in range(N)]


def init_cores(seed, K, ranks, tensor_id=0):
    """N(0,1) initial cores (R_n, K_n, R_{n+1}) for TR-ALS (random initialisation)."""
    return tr_cores(seed, K, ranks, tensor_id, tag=17)


def gaussian_kernel1d(sigma, truncate=4.0):
    """Normalised sampled Gaussian, radius round(truncate*sigma)."""
    rad = int(truncate * sigma + 0.5)
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def smooth_along(a, axis, sigma):
    """Filter ``a`` along ``axis`` with the normalised Gaussian, 'reflect' boundary
    (d c b a | a b c d | d c b a)."""
    w = gaussian_kernel1d(sigma)
    rad = (len(w) - 1) // 2
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, -1)
    n = a.shape[-1]
    idx = np.arange(-rad, n + rad)
    period = 2 * n
    m = np.mod(idx, period)
    m = np.where(m >= n, period - 1 - m, m)
    ap = a[..., m]
    out = np.zeros_like(a)
    for t in range(len(w)):
        out += w[t] * ap[..., t:t + n]
    return np.moveaxis(out, -1, axis)


def _merge(cores, device, dtype):
    """Merge consecutive cores into one (R_first, prod I, R_last) tensor."""
    T = torch.as_tensor(cores[0], device=device, dtype=dtype)
    for G in cores[1:]:
        Gt = torch.as_tensor(G, device=device, dtype=dtype)
        Ra, I, Rb = T.shape
        T = (T.reshape(Ra * I, Rb) @ Gt.reshape(Gt.shape[0], -1)).reshape(Ra, I * Gt.shape[1], Gt.shape[2])
    return T


def tr_signal(cores, device="cpu", dtype=torch.float64):
    """S = Psi(cores) as a dense torch tensor of shape (I_1, ..., I_N)."""
    dims = [g.shape[1] for g in cores]
    N = len(cores)
    h = max(1, N // 2)
    L = _merge(cores[:h], device, torch.float64)      # R1 x IL x Rh
    Rm = _merge(cores[h:], device, torch.float64)     # Rh x IR x R1
    R1, IL, Rh = L.shape
    A = L.permute(1, 0, 2).reshape(IL, R1 * Rh)                 # [il, (a, b)]
    B = Rm.permute(2, 0, 1).reshape(R1 * Rh, Rm.shape[1])       # [(a, b), ir]
    S = (A @ B).reshape(dims)
    return S.to(dtype)


_PH_M0, _PH_M1 = 0xD2511F53, 0xCD9E8D57
_PH_W0, _PH_W1 = 0x9E3779B9, 0xBB67AE85
_U32 = 0xFFFFFFFF
NOISE_STREAM = 3 << 24


def _philox_words(c, stream, tensor_id, seed):
    """Philox4x32-10 of the counters (c lo, c hi, stream, tensor_id) under key ``seed``.
    ``c`` is an int64 torch tensor of call indices; returns four int64 tensors of 32-bit
    words.  Products of two 32-bit words are formed in int64, which wraps modulo 2^64, so
    the low and high halves are exact."""
    c0 = c & _U32
    c1 = (c >> 32) & _U32
    c2 = torch.full_like(c, stream & _U32)
    c3 = torch.full_like(c, tensor_id & _U32)
    k0, k1 = seed & _U32, (seed >> 32) & _U32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PH_W0) & _U32
            k1 = (k1 + _PH_W1) & _U32
        p0 = c0 * _PH_M0
        p1 = c2 * _PH_M1
        c0, c1, c2, c3 = (((p1 >> 32) & _U32) ^ c1 ^ k0, p1 & _U32,
                          ((p0 >> 32) & _U32) ^ c3 ^ k1, p0 & _U32)
    return c0, c1, c2, c3


def _box_muller(wa, wb):
    ua = (wa.double() + 0.5) * 2.0 ** -32
    ub = (wb.double() + 0.5) * 2.0 ** -32
    r = torch.sqrt(-2.0 * torch.log(ua))
    t = (2.0 * np.pi) * ub
    return r * torch.cos(t), r * torch.sin(t)


def stream_normals(seed, stream, tensor_id, e):
    """FP64 N(0,1) samples for the stream elements ``e`` (int64 torch tensor, any shape)."""
    w = _philox_words(e >> 2, stream, tensor_id, seed)
    z01 = _box_muller(w[0], w[1])
    z23 = _box_muller(w[2], w[3])
    lane = e & 3
    return torch.where(lane == 0, z01[0], torch.where(lane == 1, z01[1],
                       torch.where(lane == 2, z23[0], z23[1])))


def _stream_run(seed, stream, tensor_id, e0, count, device):
    """FP64 stream elements [e0, e0 + count): one generator call per four elements."""
    c = torch.arange(e0 >> 2, ((e0 + count - 1) >> 2) + 1, dtype=torch.int64, device=device)
    w = _philox_words(c, stream, tensor_id, seed)
    z01 = _box_muller(w[0], w[1])
    z23 = _box_muller(w[2], w[3])
    z = torch.stack([z01[0], z01[1], z23[0], z23[1]], dim=1).reshape(-1)
    off = e0 - 4 * (e0 >> 2)
    return z[off:off + count]


def noise_block(seed, tensor_id, full_dims, dims, device="cpu", out=None, scale=1.0):
    """Noise of the leading ``dims`` block of a tensor of shape ``full_dims``: element
    (i_1..i_N) is stream element e = row-major index of (i_1..i_N) in ``full_dims``.
    Returns FP64 ``scale`` * noise, or adds it into ``out`` (FP64, shape ``dims``).  Built in
    slabs of the first index to bound temporary memory."""
    dims = [int(d) for d in dims]
    full = [int(d) for d in full_dims]
    N = len(dims)
    strides = [1] * N
    for n in range(N - 2, -1, -1):
        strides[n] = strides[n + 1] * full[n + 1]
    if out is None:
        out = torch.zeros(dims, dtype=torch.float64, device=device)
    rest = int(np.prod(dims[1:])) if N > 1 else 1
    i0_chunk = max(1, (1 << 24) // max(rest, 1))
    contiguous = dims[1:] == full[1:]  # each slab of the first index is one run of the stream
    off = None
    if not contiguous:
        # offsets of the block's elements inside one slab of the first index
        off = torch.zeros([1] * N, dtype=torch.int64, device=device)
        for n in range(1, N):
            shp = [1] * N
            shp[n] = dims[n]
            off = off + (torch.arange(dims[n], dtype=torch.int64, device=device) * strides[n]).reshape(shp)
    for a in range(0, dims[0], i0_chunk):
        b = min(dims[0], a + i0_chunk)
        if contiguous:
            z = _stream_run(seed, NOISE_STREAM, tensor_id, a * strides[0], (b - a) * rest, device)
            z = z.reshape([b - a] + dims[1:])
        else:
            i0 = torch.arange(a, b, dtype=torch.int64, device=device).reshape([b - a] + [1] * (N - 1))
            z = stream_normals(seed, NOISE_STREAM, tensor_id, i0 * strides[0] + off)
        out[a:b].add_(z, alpha=scale)
    return out


def tr_norm2(cores):
    """||Psi(cores)||_F^2 in closed form: trace of the product of the transfer matrices
    E_n = sum_i G_n(i) (x) G_n(i) (FP64)."""
    E = None
    for G in cores:
        G = np.asarray(G, dtype=np.float64)
        En = np.einsum("aib,cid->acbd", G, G).reshape(G.shape[0] ** 2, G.shape[2] ** 2)
        E = En if E is None else E @ En
    return float(np.trace(E))


def noise_sigma(signal_norm2, numel, snr_db):
    """sigma with sigma^2 numel = ||S||^2 10^(-snr/10)."""
    return (signal_norm2 * 10.0 ** (-snr_db / 10.0) / numel) ** 0.5


@dataclass
class Workload:
    """One synthetic decomposition problem."""
    name: str
    dims: List[int]
    ranks: List[int]          # TR-rank of the generator and of the decomposition
    K: List[int]              # projection size per mode
    q: int                    # power iterations
    sweeps: int               # TR-ALS sweeps
    snr_db: Optional[float]
    seed: int
    smooth_sigma: Optional[float] = None   # Gaussian smoothing of the first two cores
    rescale01: bool = False
    tol: float = 0.0
    tensor_id: int = 0
    full_dims: Optional[List[int]] = None  # this is the leading block of a tensor of these dims
    gen_ranks: Optional[List[int]] = None  # TR-rank of the generator when it differs from ranks
    smooth_modes: int = 2                  # leading modes whose cores are smoothed

    def numel(self):
        return int(np.prod(self.dims))


def small_fp64(seed_offset=1):
    """Order-4 20^4 FP64, rank 3, 40 dB, K=8, q=0, TR-ALS rank 3, 20 sweeps."""
    return Workload("small-20^4-fp64", [20] * 4, [3] * 4, [8] * 4, 0, 20, 40.0, BASE_SEED + seed_offset)


def dense_200(I=200, seed_offset=2):
    """Order-4 I^4 FP32 (200^4 = 6.4 GB), rank 6, 30 dB, K=20, q=1, TR-ALS rank 6, 30 sweeps."""
    return Workload(f"dense-{I}^4", [I] * 4, [6] * 4, [20] * 4, 1, 30, 30.0, BASE_SEED + seed_offset)


def dense_200_block(block=64, I=200, seed_offset=2):
    """The leading block^4 block of the dense I^4 workload (same cores, noise and sigma), with
    the same method parameters: the sample on which the oracle runs beside the GPU."""
    w = dense_200(I, seed_offset)
    w.name = f"dense-{I}^4-block-{block}^4"
    w.full_dims = list(w.dims)
    w.dims = [block] * 4
    return w


def hsi_shaped(scale=1, seed_offset=3):
    """1024x1024x256 FP32, rank 10, smooth spatial cores (sigma 8), [0,1], 30 dB,
    K=(60,60,40), TR-ALS rank 10, 30 sweeps.  ``scale`` divides the sizes for tests."""
    d = [1024 // scale, 1024 // scale, 256 // scale]
    K = [min(60, d[0]), min(60, d[1]), min(40, d[2])]
    return Workload(f"hsi-{d[0]}x{d[1]}x{d[2]}", d, [10] * 3, K, 0, 30, 30.0, BASE_SEED + seed_offset,
                    smooth_sigma=8.0 / scale, rescale01=True)


def rgb_shaped(I=1024, K=100, seed_offset=6):
    """Stand-in for the simulation's RGB image (Sec. 4.1): I x I x 3 FP32 from TR cores of rank
    12 whose two spatial cores are smoothed (sigma 8 at I = 1024), rescaled to [0, 1], 30 dB;
    projection K x K x 3 (the colour mode is kept); TR-ALS rank 10, 50 sweeps."""
    return Workload(f"rgb-{I}x{I}x3-K{K}", [I, I, 3], [10] * 3, [K, K, 3], 0, 50, 30.0,
                    BASE_SEED + seed_offset, smooth_sigma=8.0 * I / 1024, rescale01=True,
                    gen_ranks=[12] * 3)


def images_shaped(kind="cifar", seed_offset=7):
    """Stand-ins for the image-collection compression experiment (Sec. 4.2): 32 x 32 x 3 x 50000
    ("cifar") or 32 x 32 x 3 x 72 x 100 ("coil") FP32 from rank-8 TR cores with smooth spatial
    cores (sigma 2), rescaled to [0, 1], 30 dB; only the long sample modes are projected
    (K = 200 for the 50000 images, K = 64 for the 100 objects); TR-ALS rank 8, 30 sweeps."""
    if kind == "cifar":
        dims, K = [32, 32, 3, 50000], [32, 32, 3, 200]
    else:
        dims, K = [32, 32, 3, 72, 100], [32, 32, 3, 72, 64]
    return Workload(f"{kind}-" + "x".join(map(str, dims)), dims, [8] * len(dims), K, 0, 30, 30.0,
                    BASE_SEED + seed_offset, smooth_sigma=2.0, rescale01=True)


def hsi_small_shaped(snr_db=20.0, seed_offset=8):
    """Stand-in for the HSI reconstruction experiment (Sec. 4.3): 200 x 200 x 80 FP32 from
    rank-10 TR cores with smooth spatial cores (sigma 2), rescaled to [0, 1], noise at
    ``snr_db`` (None: noise-free); projection 100 x 100 x 6; TR-ALS rank 10, 30 sweeps."""
    tag = "clean" if snr_db is None else f"{snr_db:g}dB"
    return Workload(f"hsi-200x200x80-{tag}", [200, 200, 80], [10] * 3, [100, 100, 6], 0, 30,
                    snr_db, BASE_SEED + seed_offset, smooth_sigma=2.0, rescale01=True)


def warm_start_128(I=128, seed_offset=5):
    """128^4 FP32, rank 4, 35 dB, K=12, q=0; sweeps until the error changes by < 1e-4."""
    return Workload(f"warm-{I}^4", [I] * 4, [4] * 4, [12] * 4, 0, 100, 35.0, BASE_SEED + seed_offset, tol=1e-4)


def batched_uneven(count=512, seed_offset=4, lo=16, hi=96):
    """``count`` order-4 tensors, each I_n ~ U{lo..hi}, rank R ~ U{2..6}, K = 2R+4, 35 dB, 20 sweeps."""
    rng = _rng(BASE_SEED + seed_offset, 0, 99)
    out = []
    for t in range(count):
        dims = [int(x) for x in rng.integers(lo, hi + 1, size=4)]
        R = int(rng.integers(2, 7))
        K = [min(2 * R + 4, d) for d in dims]
        out.append(Workload(f"batched-{t}", dims, [R] * 4, K, 0, 20, 35.0, BASE_SEED + seed_offset,
                            tensor_id=t))
    return out


def make_tensor(w: Workload, device="cpu", dtype=torch.float64, clean=None):
    """Synthetic X for workload ``w``; returns (X, generating cores of X's own shape).

    The signal and the noise are formed in FP64 and rounded once to ``dtype``.  A block
    workload (``w.full_dims``) draws the cores of the full tensor, keeps their leading
    slices, and takes sigma and the noise of the full tensor, so X is exactly the leading
    block of the full tensor's X.  With ``clean`` a list, the noise-free signal (after any
    rescale, in ``dtype``) is appended to it."""
    full = list(w.full_dims) if w.full_dims else list(w.dims)
    cores = tr_cores(w.seed, full, w.gen_ranks or w.ranks, w.tensor_id)
    if w.smooth_sigma:
        cores = [smooth_along(c, 1, w.smooth_sigma) if n < w.smooth_modes else c
                 for n, c in enumerate(cores)]
    block = [c[:, :d, :] for c, d in zip(cores, w.dims)]
    S = tr_signal(block, device, torch.float64)
    if w.rescale01:
        if w.full_dims:
            raise ValueError("a rescaled workload has no block form")
        lo, hi = torch.min(S), torch.max(S)
        S = (S - lo) / (hi - lo)
        s_norm2 = float(torch.sum(S * S))
    else:
        s_norm2 = tr_norm2(cores)
    if clean is not None:
        clean.append(S.clone() if dtype == torch.float64 else S.to(dtype))
    if w.snr_db is not None:
        sigma = noise_sigma(s_norm2, int(np.prod(full)), w.snr_db)
        noise_block(w.seed, w.tensor_id, full, w.dims, device, out=S, scale=sigma)
    X = S if dtype == torch.float64 else S.to(dtype)
    return X, block


def make_init(w: Workload):
    """Random N(0,1) TR-ALS initial cores for ``w`` (shapes R x min(K, I) x R)."""
    Keff = [min(k, d) for k, d in zip(w.K, w.dims)]
    return init_cores(w.seed, Keff, w.ranks, w.tensor_id)


def sparse_tr(seed, dims, ranks, nnz, snr_db=30.0, alpha=0.8, tensor_id=0):
    """A sparse tensor: ``nnz`` distinct coordinates whose index along each mode follows a
    power law (P(i) ~ (rank of i)^-alpha over a seeded permutation of the mode, the skewed
    degree distribution of sparse count-like tensors), valued by a rank-``ranks`` TR model at
    those coordinates plus Gaussian noise at ``snr_db`` (None: none).  Returns (indices
    int64 nnz x N, values FP64, cores); entries are in the order they were first drawn."""
    rng = _rng(seed, tensor_id, 23)
    N = len(dims)
    size = int(np.prod([int(d) for d in dims], dtype=np.float64))
    nnz = int(min(nnz, size))
    pmfs, perms = [], []
    for d in dims:
        w = np.arange(1, int(d) + 1, dtype=np.float64) ** (-alpha)
        pmfs.append(w / w.sum())
        perms.append(rng.permutation(int(d)))
    chunks, have = [], np.zeros(0, dtype=np.int64)
    count = 0
    while count < nnz:
        draw = np.stack([perms[m][rng.choice(int(dims[m]), size=2 * nnz, p=pmfs[m])]
                         for m in range(N)], axis=1).astype(np.int64)
        keys = np.ravel_multi_index(tuple(draw.T), tuple(int(d) for d in dims))
        _, first = np.unique(keys, return_index=True)
        first = np.sort(first)                        # first occurrences, in drawn order
        first = first[~np.isin(keys[first], have)]    # not taken in an earlier round
        first = first[:nnz - count]
        chunks.append(draw[first])
        have = np.concatenate([have, keys[first]])
        count += len(first)
    idx = np.concatenate(chunks).reshape(nnz, N)
    cores = tr_cores(seed, dims, ranks, tensor_id, tag=29)
    T = cores[0][:, idx[:, 0], :].transpose(1, 0, 2)           # nnz x R_1 x R_2
    for n in range(1, N):
        T = np.matmul(T, cores[n][:, idx[:, n], :].transpose(1, 0, 2))
    vals = np.trace(T, axis1=1, axis2=2)
    if snr_db is not None and nnz > 0:
        sigma = np.linalg.norm(vals) / np.sqrt(nnz) * 10.0 ** (-snr_db / 20.0)
        vals = vals + sigma * rng.standard_normal(nnz)
    return idx, vals, cores
