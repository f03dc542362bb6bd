"""Brute-force pins of the Sec. 2 definitions on tiny tensors."""
import itertools

import numpy as np
import pytest

from oracle import tensor as T


def rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def test_unfold_bruteforce():
    X = rand((3, 4, 5, 2))
    for n in range(4):
        U = T.unfold(X, n)
        others = [i for i in range(4) if i != n]
        for idx in itertools.product(*[range(s) for s in X.shape]):
            j = 0
            for m in others:
                j = j * X.shape[m] + idx[m]
            assert U[idx[n], j] == X[idx]
        np.testing.assert_array_equal(T.fold(U, n, X.shape), X)


def test_unfold_tr_bruteforce():
    X = rand((3, 4, 5))
    N = 3
    for n in range(N):
        U = T.unfold_tr(X, n)
        for idx in itertools.product(*[range(s) for s in X.shape]):
            j = 0
            for t in range(1, N):
                m = (n + t) % N
                j = j * X.shape[m] + idx[m]
            assert U[idx[n], j] == X[idx]


def test_mode_product_bruteforce():
    X = rand((3, 4, 5))
    for n in range(3):
        U = rand((2, X.shape[n]), 1)
        Y = T.mode_product(X, U, n)
        for idx in itertools.product(*[range(s) for s in Y.shape]):
            s = 0.0
            for i in range(X.shape[n]):
                src = list(idx)
                src[n] = i
                s += X[tuple(src)] * U[idx[n], i]
            assert abs(Y[idx] - s) < 1e-12
        # (X x_n U)_(n) = U X_(n)
        np.testing.assert_allclose(T.unfold(Y, n), U @ T.unfold(X, n), atol=1e-12)


def _cores(dims, ranks, seed=3):
    rng = np.random.default_rng(seed)
    N = len(dims)
    return [rng.standard_normal((ranks[n], dims[n], ranks[(n + 1) % N])) for n in range(N)]


def test_tr_full_is_trace_of_slices():
    dims, ranks = [3, 4, 2, 3], [2, 3, 1, 2]
    G = _cores(dims, ranks)
    X = T.tr_full(G)
    assert X.shape == tuple(dims)
    for idx in itertools.product(*[range(s) for s in dims]):
        M = np.eye(ranks[0])
        for n in range(4):
            M = M @ G[n][:, idx[n], :]
        assert abs(X[idx] - np.trace(M)) < 1e-12


def test_tr_full_cyclic_shift_invariance():
    # trace is invariant under cyclic shift of the cores (with the modes shifted)
    dims, ranks = [3, 4, 5], [2, 3, 2]
    G = _cores(dims, ranks)
    X = T.tr_full(G)
    Xs = T.tr_full(G[1:] + G[:1])
    np.testing.assert_allclose(np.transpose(Xs, (2, 0, 1)), X, atol=1e-12)


@pytest.mark.parametrize("N", [3, 4])
def test_eq2_tr_unfolding_identity(N):
    dims = [3, 4, 2, 3][:N]
    ranks = [2, 3, 2, 4][:N]
    G = _cores(dims, ranks)
    X = T.tr_full(G)
    for n in range(N):
        S = T.subchain(G, n)
        assert S.shape == (ranks[(n + 1) % N], int(np.prod(dims)) // dims[n], ranks[n])
        lhs = T.unfold_tr(X, n)
        rhs = T.core_unfold2(G[n]) @ T.subchain_unfold2(S).T
        np.testing.assert_allclose(lhs, rhs, atol=1e-11)


def test_tr_norm_transfer_matrices():
    # ||Psi(G)||^2 = Trace(prod_n E_n), E_n = sum_i G_n(i) (x) G_n(i)  (closed form)
    dims, ranks = [4, 3, 5, 2], [2, 3, 2, 2]
    G = _cores(dims, ranks)
    E = [sum(np.kron(g[:, i, :], g[:, i, :]) for i in range(g.shape[1])) for g in G]
    M = E[0]
    for e in E[1:]:
        M = M @ e
    assert abs(np.trace(M) - T.frob(T.tr_full(G)) ** 2) < 1e-9 * np.trace(M)


def test_core_fold_roundtrip():
    g = rand((2, 5, 3))
    np.testing.assert_array_equal(T.core_fold2(T.core_unfold2(g), 2, 3), g)
