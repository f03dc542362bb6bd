"""Pins of the oracle's projection variants (Khatri-Rao test matrices, the sequential reading of
Alg. 1 step 7) against what the definitions and the mathematics fix."""
import itertools

import numpy as np
import pytest

from oracle import philox, rtr as orc
from oracle.tensor import unfold, mode_product


def tucker(dims, ranks, seed):
    """A tensor of multilinear rank ``ranks``: a Gaussian core times Gaussian factors."""
    rng = np.random.default_rng(seed)
    T = rng.standard_normal(ranks)
    for n, (d, r) in enumerate(zip(dims, ranks)):
        T = mode_product(T, rng.standard_normal((d, r)), n)
    return T


def test_khatri_rao_entrywise():
    """Entry (j, k) is the product of the factor entries of the other modes' indices, with j the
    row-major index of those indices (first other mode slowest): explicit loops."""
    dims, n, K, seed, tid = (3, 4, 2, 5), 1, 3, 77, 2
    M = orc.khatri_rao_test_matrix(seed, n, dims, K, tid)
    F = {m: philox.normals(seed, philox.stream_word(philox.TAG_KR, n, m), tid, 0, dims[m] * K)
         for m in (0, 2, 3)}
    assert M.shape == (3 * 2 * 5, K)
    j = 0
    for i0, i2, i3 in itertools.product(range(3), range(2), range(5)):
        for k in range(K):
            want = F[0][i0 * K + k] * F[2][i2 * K + k] * F[3][i3 * K + k]
            assert M[j, k] == want
        j += 1


def test_khatri_rao_factors_are_distinct_streams():
    """Each (mode, factor) pair draws its own stream: no two factors share values."""
    dims, K = (6, 7, 8), 4
    a = orc.khatri_rao_test_matrix(3, 0, dims, K)
    b = orc.khatri_rao_test_matrix(3, 1, dims, K)
    assert a.shape == (56, K) and b.shape == (48, K)
    f01 = philox.normals(3, philox.stream_word(philox.TAG_KR, 0, 1), 0, 0, 7 * K)
    f10 = philox.normals(3, philox.stream_word(philox.TAG_KR, 1, 0), 0, 0, 6 * K)
    assert not np.any(np.isin(f01, f10))


def test_khatri_rao_moments():
    """Kronecker structure: the mean square of each column is the product of the factors'
    mean squares (exactly); the factors themselves are N(0,1) (mean 0, variance 1)."""
    dims, K, seed = (2, 60, 70), 48, 11
    M = orc.khatri_rao_test_matrix(seed, 0, dims, K)
    assert M.shape == (4200, K)
    F = [philox.normals(seed, philox.stream_word(philox.TAG_KR, 0, m), 0, 0, dims[m] * K)
         .reshape(dims[m], K) for m in (1, 2)]
    want = np.mean(F[0] ** 2, axis=0) * np.mean(F[1] ** 2, axis=0)
    assert np.allclose(np.mean(M ** 2, axis=0), want, rtol=1e-12, atol=0)
    allf = np.concatenate([f.ravel() for f in F])
    assert abs(allf.mean()) < 5 / np.sqrt(allf.size)
    assert abs(allf.var() - 1.0) < 5 * np.sqrt(2.0 / allf.size)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_khatri_rao_captures_low_rank_range(n):
    """For an unfolding of rank r <= K the structured sketch spans its range exactly."""
    X = tucker((12, 10, 9), (3, 4, 2), seed=5)
    Q = orc.range_basis(X, n, 6, seed=13, test="khatri_rao")
    A = unfold(X, n)
    assert np.linalg.norm(A - Q @ (Q.T @ A)) < 1e-11 * np.linalg.norm(A)
    assert np.max(np.abs(Q.T @ Q - np.eye(6))) < 1e-13


def test_sequential_first_mode_is_the_independent_one():
    X = np.random.default_rng(1).standard_normal((9, 8, 7))
    Qs, _ = orc.sequential_bases(X, (4, 3, 3), seed=21)
    assert np.array_equal(Qs[0], orc.range_basis(X, 0, 4, seed=21))


def test_sequential_kept_modes_reduce_to_independent():
    """When modes 1..n-1 are kept (K >= I), the tensor mode n sees is X itself."""
    X = np.random.default_rng(2).standard_normal((5, 6, 9))
    Qs, P = orc.sequential_bases(X, (5, 6, 4), seed=8)
    assert np.allclose(Qs[2], orc.range_basis(X, 2, 4, seed=8), atol=1e-13, rtol=0)
    assert np.allclose(P, orc.compress(X, Qs), atol=1e-12, rtol=0)


def test_sequential_mode_two_sees_the_compressed_tensor():
    """Mode 2's basis is the QR of (X x_1 Q_1^T)_(2) times the Gaussian of that unfolding's
    width, not of X's (brute force on the explicit intermediate)."""
    X = np.random.default_rng(3).standard_normal((10, 8, 6))
    Qs, _ = orc.sequential_bases(X, (4, 3, 6), seed=5)
    T = np.einsum("ik,ijl->kjl", Qs[0], X)          # X x_1 Q_1^T by explicit contraction
    A = T.transpose(1, 0, 2).reshape(8, 4 * 6)       # its mode-2 unfolding
    M = orc.gaussian_test_matrix(5, 1, 24, 3)
    Q, R = np.linalg.qr(A @ M)
    Q = Q * np.sign(np.diag(R))[None, :]
    assert np.allclose(Qs[1], Q, atol=1e-12, rtol=0)


def test_sequential_exact_recovery():
    """A tensor of multilinear rank (2, 3, 2) is reproduced exactly from P and the bases when
    K_n >= rank_n."""
    X = tucker((11, 12, 10), (2, 3, 2), seed=9)
    Qs, P = orc.sequential_bases(X, (3, 3, 3), seed=4)
    Y = P
    for n, Q in enumerate(Qs):
        Y = mode_product(Y, Q, n)
    assert np.linalg.norm(Y - X) < 1e-11 * np.linalg.norm(X)
