"""Pins of the coordinate-list oracle (oracle/sparse.py) against definitions it does not use
itself: explicit loops over tiny tensors, the dense oracle on the densified tensor, the
Pythagorean identity of an orthogonal projection, and the linearity that makes repeated
coordinates add."""
import itertools

import numpy as np

from oracle import rtr as orc, sparse as osp
from oracle.tensor import unfold
import workloads as W


def tiny(seed=3, dims=(5, 4, 3, 6), nnz=25, dup=True):
    rng = np.random.default_rng(seed)
    idx = np.stack([rng.integers(0, d, nnz) for d in dims], axis=1).astype(np.int64)
    if dup:
        idx[-1] = idx[0]
    return idx, rng.standard_normal(nnz), dims


def test_densify_adds_repeats_and_matches_a_loop():
    idx, val, dims = tiny()
    X = osp.coo_to_dense(idx, val, dims)
    ref = np.zeros(dims)
    for c, v in zip(idx, val):
        ref[tuple(c)] = ref[tuple(c)] + v
    assert np.array_equal(X, ref)
    assert np.isclose(X[tuple(idx[0])], val[0] + val[-1], rtol=1e-15)


def test_column_index_is_the_unfolding_column():
    dims = (3, 4, 2, 5)
    X = np.arange(np.prod(dims), dtype=np.float64).reshape(dims)
    for n in range(4):
        A = unfold(X, n)
        for c in itertools.product(*[range(d) for d in dims]):
            assert A[c[n], osp.column_index(c, n, dims)] == X[c]


def test_sketch_loop_equals_dense_definition():
    idx, val, dims = tiny()
    X = osp.coo_to_dense(idx, val, dims)
    for n in range(len(dims)):
        K = 3
        J = int(np.prod([d for m, d in enumerate(dims) if m != n]))
        Y = unfold(X, n) @ orc.gaussian_test_matrix(9, n, J, K, 2)
        assert np.allclose(osp.sketch_loop(idx, val, dims, n, K, seed=9, tensor_id=2), Y,
                           rtol=1e-13, atol=1e-13)


def test_compress_loop_equals_dense_definition():
    idx, val, dims = tiny()
    rng = np.random.default_rng(4)
    Qs = [np.linalg.qr(rng.standard_normal((d, min(d, 3))))[0] for d in dims]
    X = osp.coo_to_dense(idx, val, dims)
    P = osp.compress(idx, val, dims, Qs)
    assert np.allclose(osp.compress_loop(idx, val, Qs), P, rtol=1e-13, atol=1e-13)
    # brute force over every entry of P
    Pb = np.zeros(P.shape)
    for k in itertools.product(*[range(s) for s in P.shape]):
        Pb[k] = sum(X[c] * np.prod([Qs[m][c[m], k[m]] for m in range(4)])
                    for c in itertools.product(*[range(d) for d in dims]))
    assert np.allclose(Pb, P, rtol=1e-12, atol=1e-12)


def test_range_basis_spans_the_sketch_and_pythagoras():
    idx, val, dims = tiny(nnz=40, dup=False)
    X = osp.coo_to_dense(idx, val, dims)
    Qs = [osp.range_basis(idx, val, dims, n, 2, seed=5) for n in range(4)]
    for n, Q in enumerate(Qs):
        Y = osp.sketch_loop(idx, val, dims, n, 2, seed=5)
        assert np.allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
        assert np.allclose(Q @ (Q.T @ Y), Y, atol=1e-12)
    P = osp.compress(idx, val, dims, Qs)
    XP = P
    for n, Q in enumerate(Qs):
        XP = np.moveaxis(np.tensordot(Q, XP, axes=(1, n)), 0, n)
    # orthogonal projection: ||X - X x Q Q^T||^2 = ||X||^2 - ||P||^2
    assert np.isclose(np.sum((X - XP) ** 2), np.sum(X ** 2) - np.sum(P ** 2), rtol=1e-12)


def test_linear_in_the_values_so_repeats_equal_their_sum():
    idx, val, dims = tiny(dup=False)
    idx2 = np.concatenate([idx, idx[:5]])
    val2 = np.concatenate([val * 0.25, val[:5]])
    # entries 0..4 carry 0.25 v + v, the others 0.25 v
    ref = val * 0.25
    ref[:5] += val[:5]
    for n in range(4):
        assert np.allclose(osp.sketch_loop(idx2, val2, dims, n, 2, seed=1),
                           osp.sketch_loop(idx, ref, dims, n, 2, seed=1), atol=1e-13)


def test_sparse_workload_is_seeded_distinct_and_valued_by_the_model():
    i1, v1, c1 = W.sparse_tr(7, (30, 20, 10), (2, 3, 2), 500, snr_db=None)
    i2, v2, _ = W.sparse_tr(7, (30, 20, 10), (2, 3, 2), 500, snr_db=None)
    assert np.array_equal(i1, i2) and np.array_equal(v1, v2)
    assert len({tuple(r) for r in i1}) == 500
    from oracle.tensor import tr_full
    S = tr_full(c1)
    assert np.allclose(v1, S[tuple(i1.T)], rtol=1e-12, atol=1e-12)
