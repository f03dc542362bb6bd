"""GPU TR-SVD (Alg. 1 step 9, rTR-SVD variant) against the FP64 oracle, through the C ABI.

Cores are compared through Psi (singular vectors carry a sign freedom), ranks exactly, and
the reported error against ||P - Psi(Z)|| computed on the host; the error bound
||P - Psi(Z)|| <= eps ||P|| holds whenever no rank was capped.
"""
import numpy as np
import pytest
import torch

import paper_1901_01652_amd as rt
from oracle import rtr as orc, tensor as ot

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    hd = rt.Handle(0)
    yield hd
    hd.close()


def say(*a):
    print(*a, flush=True)


def low_rank_plus_noise(dims, R, noise, seed):
    """A TR tensor of rank R (N(0,1) cores) plus i.i.d. noise of relative size ``noise``."""
    rng = np.random.default_rng(seed)
    N = len(dims)
    cores = [rng.standard_normal((R, dims[n], R)) for n in range(N)]
    S = ot.tr_full(cores)
    E = rng.standard_normal(dims)
    return S + noise * np.linalg.norm(S) / np.linalg.norm(E) * E


def run(h, P, caps, eps):
    Pd = torch.as_tensor(P).to(DEV)
    Z, ranks, err = rt.rtr_decompose_svd(h, Pd, caps, eps)
    bits = rt.rtr_status_sync(h)
    ranks = [int(r) for r in ranks.cpu()]
    cores = [c.cpu().numpy() for c in rt.svd_cores(Z, ranks, P.shape, caps)]
    return cores, ranks, float(err.cpu()[0]), bits


@pytest.mark.parametrize("dims,R,noise,eps", [
    ((8, 9, 7, 6), 2, 0.05, 0.15),
    ((8, 9, 7, 6), 2, 0.05, 0.03),
    ((8, 9, 7, 6), 2, 0.05, 0.30),
    ((12, 10, 11), 3, 0.02, 0.10),
    ((20, 20, 20, 20), 3, 0.03, 0.15),   # the dense 200^4 workload's P shape
    ((30, 3, 4), 2, 0.05, 0.10),         # first step tall: Gram of the columns
    ((5, 4, 6, 3, 4), 2, 0.05, 0.12),    # order 5
    ((40, 60), 6, 0.05, 0.10),           # order 2: the truncated SVD of a matrix
])
def test_tr_svd_matches_oracle(h, dims, R, noise, eps):
    say("tr-svd", dims, R, noise, eps)
    P = low_rank_plus_noise(dims, R, noise, seed=sum(dims) + R)
    caps = [32] * len(dims)
    cores, ranks, err, bits = run(h, P, caps, eps)
    Zo, ranks_o = orc.tr_svd(P, eps)
    assert bits == 0
    assert ranks == list(ranks_o), (ranks, ranks_o)
    Psi, Psi_o = ot.tr_full(cores), ot.tr_full(Zo)
    assert np.linalg.norm(Psi - Psi_o) / np.linalg.norm(Psi_o) < 1e-10
    explicit = np.linalg.norm(P - Psi) / np.linalg.norm(P)
    assert abs(err - explicit) <= 1e-10 * explicit + 1e-14
    assert explicit <= eps * (1 + 1e-12)


def test_tr_svd_matrix_is_eckart_young(h):
    """Order 2: TR-SVD is one truncated SVD; the error is the discarded singular energy."""
    say("tr-svd eckart-young")
    P = low_rank_plus_noise((50, 70), 5, 0.1, seed=3)
    eps = 0.08
    cores, ranks, err, _ = run(h, P, [32, 32], eps)
    s = np.linalg.svd(P, compute_uv=False)
    r = ranks[0] * ranks[1]
    assert np.sqrt(np.sum(s[r:] ** 2)) <= eps * np.linalg.norm(P)
    assert np.sqrt(np.sum(s[r - 1:] ** 2)) > eps * np.linalg.norm(P)   # minimal
    assert abs(err - np.sqrt(np.sum(s[r:] ** 2)) / np.linalg.norm(P)) < 1e-12


@pytest.mark.parametrize("dims,eps,caps", [((96, 130), 0.02, [128, 128]),
                                           ((120, 200), 0.02, [128, 128]),
                                           ((100, 150, 3), 0.01, [12, 12, 32]),
                                           ((150, 180), 0.02, [160, 160])])
def test_tr_svd_large_gram(h, dims, eps, caps):
    """The eigen-solver's three homes: Gram and eigenvectors in LDS (d = 96, the largest),
    the Gram in LDS and the eigenvectors in the workspace (d = 100, 120), both in the
    workspace (d = 150)."""
    say("tr-svd large gram", dims, eps)
    P = low_rank_plus_noise(dims, 4, 0.2, seed=11)
    cores, ranks, err, bits = run(h, P, caps, eps)
    Zo, ranks_o = orc.tr_svd(P, eps)
    assert bits == 0 and ranks == list(ranks_o), (ranks, ranks_o)
    Psi, Psi_o = ot.tr_full(cores), ot.tr_full(Zo)
    assert np.linalg.norm(Psi - Psi_o) / np.linalg.norm(Psi_o) < 1e-10


def test_tr_svd_rank_cap(h):
    """Caps below the tolerance's ranks: ranks clamped, status bit set, the reported error
    still that of the returned cores."""
    say("tr-svd caps")
    dims = (8, 9, 7, 6)
    P = low_rank_plus_noise(dims, 3, 0.05, seed=5)
    caps = [1, 2, 2, 2]
    cores, ranks, err, bits = run(h, P, caps, 0.01)
    assert bits & rt.RTR_STATUS_RANK_CAPPED
    assert all(r <= c for r, c in zip(ranks, caps))
    explicit = np.linalg.norm(P - ot.tr_full(cores)) / np.linalg.norm(P)
    assert abs(err - explicit) <= 1e-10 * explicit
    assert rt.rtr_status_sync(h) == 0


def test_tr_svd_exact_tr_tensor(h):
    """A noiseless TR tensor whose ranks TR-SVD can represent is recovered to rounding."""
    say("tr-svd exact")
    rng = np.random.default_rng(9)
    R = [2, 3, 2, 2]
    dims = (7, 8, 6, 5)
    cores = [rng.standard_normal((R[n], dims[n], R[(n + 1) % 4])) for n in range(4)]
    P = ot.tr_full(cores)
    got, ranks, err, bits = run(h, P, [8, 8, 8, 8], 1e-6)
    assert bits == 0 and ranks[0] * ranks[1] == 6
    assert np.linalg.norm(P - ot.tr_full(got)) / np.linalg.norm(P) < 1e-11
    assert err < 1e-6


def test_tr_svd_invalid(h):
    P = torch.zeros((4, 5, 6), dtype=torch.float64, device=DEV)
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose_svd(h, P, [4, 4, 4], 0.0)
    assert e.value.code == 1
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose_svd(h, P, [0, 4, 4], 0.1)
    assert e.value.code == 1
    big = torch.zeros((600, 700), dtype=torch.float64, device=DEV)
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose_svd(h, big, [32, 32], 0.1)   # Gram of 600 > 512
    assert e.value.code == 2
