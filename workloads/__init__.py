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

Noise and signal are produced with torch on the requested device; numbers are reproducible
for a given (seed, device type).  Small cases are generated on the CPU and copied.
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


def add_noise(S, snr_db, seed, tensor_id=0):
    """X = S + sigma * N(0,1) with sigma^2 numel = ||S||^2 10^(-snr/10); returns (X, sigma)."""
    if snr_db is None:
        return S.clone(), 0.0
    nS2 = float(torch.sum(S.double() ** 2))
    sigma = (nS2 * 10.0 ** (-snr_db / 10.0) / S.numel()) ** 0.5
    g = torch.Generator(device=S.device)
    g.manual_seed((int(seed) * 1000003 + int(tensor_id) * 7919 + 5) % (2 ** 63))
    E = torch.randn(S.shape, generator=g, device=S.device, dtype=S.dtype)
    E.mul_(sigma)
    E.add_(S)
    return E, sigma


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

    def numel(self):
        return int(np.prod(self.dims))


def small_fp64(seed_offset=1):
    """Order-4 20^4 FP64, rank 3, 40 dB, K=8, q=0, TR-ALS rank 3, 20 sweeps."""
    return Workload("small-20^4-fp64", [20] * 4, [3] * 4, [8] * 4, 0, 20, 40.0, BASE_SEED + seed_offset)


def dense_200(I=200, seed_offset=2):
    """Order-4 I^4 FP32 (200^4 = 6.4 GB), rank 6, 30 dB, K=20, q=1, TR-ALS rank 6, 30 sweeps."""
    return Workload(f"dense-{I}^4", [I] * 4, [6] * 4, [20] * 4, 1, 30, 30.0, BASE_SEED + seed_offset)


def hsi_shaped(scale=1, seed_offset=3):
    """1024x1024x256 FP32, rank 10, smooth spatial cores (sigma 8), [0,1], 30 dB,
    K=(60,60,40), TR-ALS rank 10, 30 sweeps.  ``scale`` divides the sizes for tests."""
    d = [1024 // scale, 1024 // scale, 256 // scale]
    K = [min(60, d[0]), min(60, d[1]), min(40, d[2])]
    return Workload(f"hsi-{d[0]}x{d[1]}x{d[2]}", d, [10] * 3, K, 0, 30, 30.0, BASE_SEED + seed_offset,
                    smooth_sigma=8.0 / scale, rescale01=True)


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


def make_tensor(w: Workload, device="cpu", dtype=torch.float64):
    """Synthetic X for workload ``w``; returns (X, generating cores)."""
    cores = tr_cores(w.seed, w.dims, w.ranks, w.tensor_id)
    if w.smooth_sigma:
        cores = [smooth_along(c, 1, w.smooth_sigma) if n < 2 else c for n, c in enumerate(cores)]
    S = tr_signal(cores, device, torch.float64 if device == "cpu" else torch.float32)
    if w.rescale01:
        lo, hi = torch.min(S), torch.max(S)
        S = (S - lo) / (hi - lo)
    S = S.to(dtype)
    X, _ = add_noise(S, w.snr_db, w.seed, w.tensor_id)
    return X, cores


def make_init(w: Workload):
    """Random N(0,1) TR-ALS initial cores for ``w`` (shapes R x min(K, I) x R)."""
    Keff = [min(k, d) for k, d in zip(w.K, w.dims)]
    return init_cores(w.seed, Keff, w.ranks, w.tensor_id)
