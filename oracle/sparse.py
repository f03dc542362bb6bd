"""Alg. 1 steps 4-7 for a tensor given by its nonzeros (coordinate list), in FP64.

The paper's conclusion (Sec. 5) names sparse tensors as future work.  Reading: the method is
unchanged; X is the sum over entries z of v_z e_{i_1(z)} (x) .. (x) e_{i_N(z)} (repeated
coordinates add), and every step applies to that X as defined for a dense one.  Each function
below takes that definition literally: densify, then the dense oracle's step, or a plain loop
over the nonzeros for the pins.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import rtr as orc


def coo_to_dense(indices, values, dims):
    """The dense tensor with values added at their coordinates (repeats add).

    Parity: pinned by an explicit loop and by repeats equal to their sum."""
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    np.add.at(X, tuple(np.asarray(indices, dtype=np.int64).T), np.asarray(values, dtype=np.float64))
    return X


def column_index(coord, n, dims):
    """Column of X_(n) holding the entry at ``coord``: the other modes' indices, row-major,
    first other mode slowest (the unfolding order of the dense oracle).

    Parity: pinned entry by entry against the dense unfolding."""
    j = 0
    for m, d in enumerate(dims):
        if m != n:
            j = j * int(d) + int(coord[m])
    return j


def sketch_loop(indices, values, dims, n, K, seed=0, tensor_id=0):
    """Y_n = X_(n) M_n (Alg. 1 steps 4-5) by a loop over the nonzeros: row i_n of Y_n gains v
    times row j_n of M_n.

    Parity: pinned against X_(n) M_n of the densified tensor and by linearity in the values."""
    dims = [int(d) for d in dims]
    J = int(np.prod([d for m, d in enumerate(dims) if m != n]))
    M = orc.gaussian_test_matrix(seed, n, J, K, tensor_id)
    Y = np.zeros((dims[n], K))
    for coord, v in zip(np.asarray(indices), np.asarray(values, dtype=np.float64)):
        Y[int(coord[n])] += v * M[column_index(coord, n, dims)]
    return Y


def compress_loop(indices, values, Qs):
    """P = X x_1 Q_1^T .. x_N Q_N^T (Eq. 3) by a loop over the nonzeros: each adds v times
    the outer product of row i_n of every Q_n.

    Parity: pinned against the dense oracle and an entry-by-entry brute force."""
    P = np.zeros(tuple(Q.shape[1] for Q in Qs))
    for coord, v in zip(np.asarray(indices), np.asarray(values, dtype=np.float64)):
        T = np.array(v)
        for Q, i in zip(Qs, coord):
            T = np.multiply.outer(T, Q[int(i)])
        P += T
    return P


def range_basis(indices, values, dims, n, K, seed=0, tensor_id=0):
    """Q_n of Alg. 1 step 6 for the tensor the coordinate list defines (no power iterations).

    Parity: orthonormal, spans the loop-formed sketch; the dense oracle's pins apply."""
    return orc.range_basis(coo_to_dense(indices, values, dims), n, K, 0, seed, tensor_id)


def compress(indices, values, dims, Qs):
    """Eq. (3) for the tensor the coordinate list defines.

    Parity: pinned by the loop and brute force above and by the Pythagorean identity."""
    return orc.compress(coo_to_dense(indices, values, dims), Qs)
