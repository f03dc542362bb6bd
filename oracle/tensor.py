"""Definitions of Sec. 2 (notation and the tensor-ring format), FP64.

Conventions (readings stated where the paper leaves a choice):
* Arrays are row-major (last index fastest); modes are 0-based in code, 1-based in the paper.
* Mode-n unfolding X_(n) (Sec. 2.1, after Kolda & Bader): rows i_n, columns run over the
  remaining indices (i_1..i_{n-1}, i_{n+1}..i_N) in row-major order.  The paper fixes only
  the row index; any column order works as long as every use agrees (Y = X_(n) M pairs each
  column with one row of M).
* TR unfolding X_<n> (Sec. 2.1): rows i_n, columns row-major over the cyclic order
  (i_{n+1}, ..., i_N, i_1, ..., i_{n-1}).
* Core G_n has shape (R_n, I_n, R_{n+1}) with R_{N+1} = R_1 (Sec. 2.2); the slice
  G_n(i_n) = G_n[:, i_n, :] is R_n x R_{n+1}.
"""
import numpy as np


def unfold(X, n):
    """Mode-n unfolding X_(n) (Sec. 2.1)."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def fold(M, n, shape):
    """Inverse of ``unfold``."""
    rest = [s for i, s in enumerate(shape) if i != n]
    return np.moveaxis(M.reshape([shape[n]] + rest), 0, n)


def unfold_tr(X, n):
    """TR unfolding X_<n> (Sec. 2.1): columns over the cyclic order after mode n."""
    N = X.ndim
    order = [(n + t) % N for t in range(N)]
    return np.transpose(X, order).reshape(X.shape[n], -1)


def mode_product(X, U, n):
    """Mode-n product X x_n U with U of shape (J, I_n) (Sec. 3.1, after Kolda & Bader):
    (X x_n U)[.., j, ..] = sum_i X[.., i, ..] U[j, i]; equivalently (X x_n U)_(n) = U X_(n)."""
    return np.moveaxis(np.tensordot(U, X, axes=(1, n)), 0, n)


def tr_full(cores):
    """Psi([G_n]) of Eq. (4): element (i_1..i_N) = Trace(G_1(i_1) ... G_N(i_N)) (Eq. 1).

    Computed by merging the cores left to right and tracing the two open rank indices."""
    T = cores[0]
    for G in cores[1:]:
        T = np.tensordot(T, G, axes=(T.ndim - 1, 0))
    return np.trace(T, axis1=0, axis2=T.ndim - 1)


def subchain(cores, n):
    """Subchain tensor G_{!=n} (Sec. 2.2): merge G_{n+1}, .., G_N, G_1, .., G_{n-1}.

    Shape (R_{n+1}, prod_{i!=n} I_i, R_n); the middle index is row-major over the cyclic
    order (i_{n+1}, ..., i_{n-1}), i.e. the column order of X_<n>."""
    N = len(cores)
    idx = [(n + t) % N for t in range(1, N)]
    T = cores[idx[0]]
    for m in idx[1:]:
        T = np.tensordot(T, cores[m], axes=(T.ndim - 1, 0))
    return T.reshape(T.shape[0], -1, T.shape[-1])


def core_unfold2(G):
    """G_{n,(2)}: (I_n, R_n R_{n+1}) with column index a*R_{n+1} + b for G[a, i, b]."""
    return np.transpose(G, (1, 0, 2)).reshape(G.shape[1], -1)


def core_fold2(W, Ra, Rb):
    """Inverse of ``core_unfold2``: (I, Ra*Rb) -> core (Ra, I, Rb)."""
    return np.transpose(W.reshape(W.shape[0], Ra, Rb), (1, 0, 2))


def subchain_unfold2(S):
    """G_{!=n,<2>}: (prod I, R_n R_{n+1}) with column a*R_{n+1} + b holding S[b, j, a], so that
    Eq. (2) reads X_<n> = core_unfold2(G_n) @ subchain_unfold2(G_{!=n}).T."""
    return np.transpose(S, (1, 2, 0)).reshape(S.shape[1], -1)


def frob(X):
    """Frobenius norm ||X||_F = sqrt(<X, X>) (Sec. 2.1)."""
    return float(np.sqrt(np.sum(np.asarray(X, dtype=np.float64) ** 2)))
