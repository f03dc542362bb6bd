"""Pins of the oracle's Algorithm 1 steps: exact recovery, closed forms, textbook limits."""
import numpy as np
import scipy.linalg
import pytest

from oracle import rtr, tensor as T
import workloads as W


def cores(dims, ranks, seed=5):
    rng = np.random.default_rng(seed)
    N = len(dims)
    return [rng.standard_normal((ranks[n], dims[n], ranks[(n + 1) % N])) for n in range(N)]


def test_qr_pos_matches_cholesky_route():
    Y = np.random.default_rng(1).standard_normal((50, 7))
    Q, R = rtr.qr_pos(Y)
    Rc = np.linalg.cholesky(Y.T @ Y).T           # upper, positive diagonal
    Qc = Y @ np.linalg.inv(Rc)
    np.testing.assert_allclose(Q, Qc, atol=1e-12)
    np.testing.assert_allclose(R, Rc, atol=1e-11)
    assert np.all(np.diag(R) >= 0)
    assert np.max(np.abs(Q.T @ Q - np.eye(7))) < 1e-13
    np.testing.assert_allclose(Q @ R, Y, atol=1e-12)


def test_gaussian_matrix_rows_keyed_by_multiindex():
    # M for mode n is indexed by the row-major multi-index of the other modes
    M = rtr.gaussian_test_matrix(3, 1, 60, 5)
    M2 = rtr.gaussian_test_matrix(3, 1, 61, 5)
    np.testing.assert_array_equal(M, M2[:60])
    assert M.shape == (60, 5)


def test_range_finder_textbook_matrix_case():
    # N = 2: Y = A M, Q = qr(Y); if K >= rank(A) then Q Q^T A = A (Halko et al. Alg. 4.1)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((40, 6)) @ rng.standard_normal((6, 50))
    Q = rtr.range_basis(A, 0, 8, 0, seed=11)
    np.testing.assert_allclose(Q @ (Q.T @ A), A, atol=1e-10)
    Q1 = rtr.range_basis(A, 1, 8, 0, seed=11)
    np.testing.assert_allclose((A @ Q1) @ Q1.T, A, atol=1e-10)


def test_power_iteration_equals_closed_form():
    # exact arithmetic: Q(q) = qr((A A^T)^q A M) whatever the re-orthonormalisation schedule
    rng = np.random.default_rng(4)
    U, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((80, 30)))
    s = 0.8 ** np.arange(30)
    A = (U * s) @ V.T
    X = A.reshape(30, 8, 10)
    K, seed = 6, 7
    M = rtr.gaussian_test_matrix(seed, 0, 80, K)
    for q in (0, 1, 2):
        Q = rtr.range_basis(X, 0, K, q, seed)
        Qc, _ = rtr.qr_pos(np.linalg.matrix_power(A @ A.T, q) @ A @ M)
        np.testing.assert_allclose(Q, Qc, atol=1e-9)


def test_power_iteration_improves_range():
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    V, _ = np.linalg.qr(rng.standard_normal((300, 60)))
    s = 1.0 / (1.0 + np.arange(60)) ** 0.5
    A = (U * s) @ V.T
    X = A.reshape(60, 20, 15)
    K = 10
    err = []
    for q in (0, 1, 3):
        Q = rtr.range_basis(X, 0, K, q, seed=3)
        err.append(np.linalg.norm(A - Q @ (Q.T @ A), 2))
    assert err[1] < err[0] and err[2] < err[1]
    assert err[2] >= s[K] * (1 - 1e-12)          # never better than sigma_{K+1}
    assert err[2] < 1.6 * s[K]


def test_exact_recovery_projection_and_compression():
    dims, ranks, K = [8, 9, 7, 8], [2, 2, 2, 2], [6, 5, 6, 4]
    G = cores(dims, ranks)
    X = T.tr_full(G)
    Qs = [rtr.range_basis(X, n, K[n], 0, seed=1) for n in range(4)]
    for n, Q in enumerate(Qs):
        assert np.max(np.abs(Q.T @ Q - np.eye(K[n]))) < 1e-13
        # X x_n Q Q^T = X
        np.testing.assert_allclose(T.mode_product(X, Q @ Q.T, n), X, atol=1e-11 * np.abs(X).max())
    P = rtr.compress(X, Qs)
    Zstar = [np.einsum("ik,aib->akb", Q, g) for Q, g in zip(Qs, G)]    # G_n x_2 Q_n^T
    np.testing.assert_allclose(P, T.tr_full(Zstar), atol=1e-10 * np.abs(P).max())
    # back-projection of the exact small cores recovers X
    np.testing.assert_allclose(T.tr_full(rtr.backproject(Zstar, Qs)), X, atol=1e-10 * np.abs(X).max())


def test_compression_mode_order_and_identity():
    rng = np.random.default_rng(8)
    X = rng.standard_normal((6, 7, 5))
    Qs = [np.linalg.qr(rng.standard_normal((d, k)))[0] for d, k in zip(X.shape, (3, 4, 2))]
    P = rtr.compress(X, Qs)
    P2 = X
    for n in (2, 0, 1):
        P2 = T.mode_product(P2, Qs[n].T, n)
    np.testing.assert_allclose(P, P2, atol=1e-12)
    np.testing.assert_allclose(rtr.compress(X, [np.eye(d) for d in X.shape]), X, atol=0)


def test_pythagorean_identity():
    # ||X - Psi(G)||^2 = ||X||^2 - ||P||^2 + ||P - Psi(Z)||^2 with G_n = Z_n x_2 Q_n
    rng = np.random.default_rng(9)
    X = rng.standard_normal((7, 6, 8))
    Qs = [np.linalg.qr(rng.standard_normal((d, k)))[0] for d, k in zip(X.shape, (4, 3, 5))]
    P = rtr.compress(X, Qs)
    Z = cores([4, 3, 5], [2, 3, 2], seed=10)
    G = rtr.backproject(Z, Qs)
    lhs = T.frob(X - T.tr_full(G)) ** 2
    rhs = T.frob(X) ** 2 - T.frob(P) ** 2 + T.frob(P - T.tr_full(Z)) ** 2
    assert abs(lhs - rhs) < 1e-10 * T.frob(X) ** 2


def test_backprojection_multilinearity():
    rng = np.random.default_rng(12)
    Z = cores([3, 4, 2, 3], [2, 2, 3, 2], seed=13)
    Qs = [rng.standard_normal((d, k)) for d, k in zip([5, 6, 4, 7], [3, 4, 2, 3])]
    lhs = T.tr_full(rtr.backproject(Z, Qs))
    rhs = T.tr_full(Z)
    for n, Q in enumerate(Qs):
        rhs = T.mode_product(rhs, Q, n)
    np.testing.assert_allclose(lhs, rhs, atol=1e-10)


def test_als_fixed_point_at_exact_cores():
    dims, ranks = [6, 5, 6, 5], [2, 2, 2, 2]
    G = cores(dims, ranks, seed=14)
    P = T.tr_full(G)
    Z, tr = rtr.tr_als(P, G, 3)
    assert tr.max() < 1e-12
    np.testing.assert_allclose(T.tr_full(Z), P, atol=1e-10)


def test_als_recovers_well_posed_tensor_from_random_init():
    dims, ranks, K = [8, 8, 8, 8], [2, 2, 2, 2], [6, 6, 6, 6]
    G = cores(dims, ranks, seed=15)
    X = T.tr_full(G)
    Z0 = cores(K, ranks, seed=16)
    out = rtr.rtr_als(X, K, Z0, sweeps=60, seed=3)
    assert out["rse"] < 1e-10
    assert out["rse_trace"][-1] < 1e-10


def test_als_monotone_per_update():
    dims, ranks = [6, 7, 5, 6], [3, 2, 3, 2]
    rng = np.random.default_rng(17)
    P = T.tr_full(cores(dims, [4, 4, 4, 4], seed=18)) + 0.1 * rng.standard_normal(dims)
    Z0 = cores(dims, ranks, seed=19)
    _, _, upd = rtr.tr_als(P, Z0, 6, record_updates=True)
    assert np.all(np.diff(upd) <= 1e-12)


def test_als_update_is_least_squares_optimum():
    dims, ranks = [5, 6, 4], [2, 3, 2]
    rng = np.random.default_rng(20)
    P = rng.standard_normal(dims)
    Z = cores(dims, ranks, seed=21)
    for n in range(3):
        Z[n] = rtr.als_update(P, Z, n)
        base = T.frob(P - T.tr_full(Z))
        for t in range(5):
            D = 1e-4 * rng.standard_normal(Z[n].shape)
            Zp = list(Z)
            Zp[n] = Z[n] + D
            assert T.frob(P - T.tr_full(Zp)) >= base - 1e-13
        # gradient of ||P - Psi||^2 w.r.t. Z_n vanishes
        B = T.subchain_unfold2(T.subchain(Z, n))
        R = T.unfold_tr(P - T.tr_full(Z), n)
        assert np.max(np.abs(R @ B)) < 1e-9 * T.frob(P) * np.abs(B).max()


def test_als_matrix_case_reaches_eckart_young():
    # N = 2: Psi is a product with inner dimension R_1 R_2; ALS converges to the truncated SVD
    rng = np.random.default_rng(22)
    U, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((25, 25)))
    s = 0.7 ** np.arange(25)
    A = (U[:, :25] * s) @ V.T
    ranks = [2, 3]
    Z0 = cores([30, 25], ranks, seed=23)
    Z, tr = rtr.tr_als(A, Z0, 200)
    r = ranks[0] * ranks[1]
    ey = np.sqrt(np.sum(s[r:] ** 2)) / np.sqrt(np.sum(s ** 2))
    assert abs(tr[-1] - ey) < 1e-8


def test_full_projection_equals_plain_tr_als():
    # K_n = I_n: Q_n = I and rTR-ALS is TR-ALS on X (the paper's "counterpart")
    rng = np.random.default_rng(24)
    X = rng.standard_normal((5, 6, 4, 5))
    ranks = [2, 2, 2, 2]
    Z0 = cores(X.shape, ranks, seed=25)
    out = rtr.rtr_als(X, list(X.shape), Z0, sweeps=5)
    Z, tr = rtr.tr_als(X, Z0, 5)
    np.testing.assert_allclose(out["rse_trace"], tr, rtol=1e-12)
    np.testing.assert_allclose(T.tr_full(out["G"]), T.tr_full(Z), atol=1e-10)


def test_als_tolerance_stop():
    rng = np.random.default_rng(26)
    P = rng.standard_normal((5, 5, 5))
    Z0 = cores([5, 5, 5], [2, 2, 2], seed=27)
    _, full = rtr.tr_als(P, Z0, 50)
    _, tr = rtr.tr_als(P, Z0, 50, tol=1e-4)
    s = len(tr)
    np.testing.assert_allclose(tr, full[:s], rtol=1e-12)
    assert abs(tr[-1] - tr[-2]) < 1e-4
    assert all(abs(full[i] - full[i - 1]) >= 1e-4 for i in range(1, s - 1))


@pytest.mark.parametrize("eps", [0.3, 0.1, 0.01])
def test_tr_svd_error_bound_and_minimal_ranks(eps):
    rng = np.random.default_rng(28)
    P = T.tr_full(cores([6, 7, 5, 6], [2, 3, 2, 3], seed=29)) + 0.05 * rng.standard_normal((6, 7, 5, 6))
    Z, ranks = rtr.tr_svd(P, eps)
    err = T.frob(P - T.tr_full(Z)) / T.frob(P)
    assert err <= eps * (1 + 1e-12)
    assert [z.shape[0] for z in Z] == ranks
    # first truncation: rank r_1 = R_1 R_2 is the smallest meeting sqrt(2) eps ||P|| / sqrt(N)
    s = np.linalg.svd(P.reshape(6, -1), compute_uv=False)
    d1 = np.sqrt(2) * eps * T.frob(P) / 2.0
    r1 = ranks[0] * ranks[1]
    assert np.sqrt(np.sum(s[r1:] ** 2)) <= d1
    if r1 > 1:
        assert np.sqrt(np.sum(s[r1 - 1:] ** 2)) > d1


def _sv_by_eigh(C):
    """Singular values of C from the symmetric eigen-solver on the smaller Gram matrix (a
    route independent of the SVD that tr_svd calls), descending."""
    G = C @ C.T if C.shape[0] <= C.shape[1] else C.T @ C
    ev = scipy.linalg.eigvalsh(G)[::-1]
    return np.sqrt(np.maximum(ev, 0.0))


@pytest.mark.parametrize("shape,ranks,noise,eps", [
    ((6, 7, 5, 6), (2, 3, 2, 3), 0.05, 0.3),
    ((6, 7, 5, 6), (2, 3, 2, 3), 0.05, 0.1),
    ((6, 7, 5, 6), (2, 3, 2, 3), 0.05, 0.02),
    ((5, 6, 4, 5, 4), (2, 2, 3, 2, 2), 0.1, 0.2),
    ((9, 8, 10), (3, 2, 4), 0.02, 0.05),
])
def test_tr_svd_every_truncation_minimal(shape, ranks, noise, eps):
    """Every truncation of TR-SVD keeps the smallest rank whose discarded singular values
    fit its budget (tail(r) <= budget < tail(r - 1)), the budgets are eps ||P|| / sqrt(N)
    (twice the energy for the first), and the final error is exactly the root sum of the
    discarded tails (the truncations are orthogonal projections onto nested subspaces)."""
    rng = np.random.default_rng(40)
    S = T.tr_full(cores(list(shape), list(ranks), seed=41))
    P = S + noise * np.std(S) * rng.standard_normal(shape)
    steps = []
    Z, R = rtr.tr_svd(P, eps, steps=steps)
    N = len(shape)
    assert len(steps) == N - 1
    nP = T.frob(P)
    lost2 = 0.0
    for k, (C, budget, r) in enumerate(steps):
        want = eps * nP / np.sqrt(N) * (np.sqrt(2.0) if k == 0 else 1.0)
        assert abs(budget - want) <= 1e-14 * want
        s = _sv_by_eigh(C)
        tail = lambda t: float(np.sqrt(np.sum(s[t:] ** 2)))
        assert tail(r) <= budget * (1 + 1e-9), (k, r, tail(r), budget)
        if r > 1:
            assert tail(r - 1) > budget * (1 - 1e-9), (k, r, tail(r - 1), budget)
        lost2 += tail(r) ** 2
    err = T.frob(P - T.tr_full(Z))
    assert abs(err - np.sqrt(lost2)) <= 1e-8 * nP
    assert err <= eps * nP * (1 + 1e-12)
    # the kept ranks are the cores' ranks (first split into R_1 R_2)
    assert steps[0][2] == R[0] * R[1]
    assert [st[2] for st in steps[1:]] == R[2:]


def test_tr_svd_tensor_train_ranks_exact():
    """With R_1 = 1 the ring is a tensor train, whose sequential unfoldings have the TT-ranks
    as exact ranks: TR-SVD at a tiny eps must return exactly those ranks."""
    G = cores([6, 7, 8, 5], [1, 3, 4, 2], seed=42)
    P = T.tr_full(G)
    Z, R = rtr.tr_svd(P, 1e-9)
    assert R == [1, 3, 4, 2]
    assert T.frob(P - T.tr_full(Z)) <= 1e-9 * T.frob(P)


def test_tr_svd_independent_of_lapack_signs(monkeypatch):
    """The split first rank makes TR-SVD depend on singular-vector signs; with the fixed
    sign rule the result is a function of P alone: random sign flips of every SVD that
    LAPACK returns change nothing, while without the rule they change the error."""
    rng = np.random.default_rng(31)
    P = T.tr_full(cores([12, 10, 11], [3, 3, 3], seed=32)) + 0.1 * rng.standard_normal((12, 10, 11))
    Z, ranks = rtr.tr_svd(P, 0.1)
    base = T.tr_full(Z)
    svd = np.linalg.svd
    flips = np.random.default_rng(33)

    def flipped_svd(C, full_matrices=False):
        U, s, Vt = svd(C, full_matrices=full_matrices)
        sg = flips.choice([-1.0, 1.0], size=len(s))
        return U * sg, s, Vt * sg[:, None]

    monkeypatch.setattr(rtr.np.linalg, "svd", flipped_svd)
    for _ in range(4):
        Z2, ranks2 = rtr.tr_svd(P, 0.1)
        assert ranks2 == ranks
        np.testing.assert_allclose(T.tr_full(Z2), base, rtol=0, atol=1e-12 * np.abs(base).max())
    # the dependence the rule removes: flip one pair of the first SVD by hand
    monkeypatch.setattr(rtr.np.linalg, "svd", svd)
    C = P.reshape(12, -1)
    U, s, Vt = rtr._svd_fixed_sign(C)
    r = ranks[0] * ranks[1]
    assert ranks[0] > 1 and r > 1
    U2, Vt2 = U.copy(), Vt.copy()
    U2[:, 1] *= -1
    Vt2[1] *= -1
    C2a = np.transpose((s[:r, None] * Vt[:r]).reshape(ranks[0], ranks[1], -1), (1, 2, 0))
    C2b = np.transpose((s[:r, None] * Vt2[:r]).reshape(ranks[0], ranks[1], -1), (1, 2, 0))
    sa = np.linalg.svd(C2a.reshape(ranks[1] * 10, -1), compute_uv=False)
    sb = np.linalg.svd(C2b.reshape(ranks[1] * 10, -1), compute_uv=False)
    assert np.max(np.abs(sa - sb)) > 1e-6 * sa[0]


def test_tr_svd_exact_for_tr_tensor():
    P = T.tr_full(cores([5, 6, 5, 4], [2, 2, 2, 2], seed=30))
    Z, ranks = rtr.tr_svd(P, 1e-10)
    assert T.frob(P - T.tr_full(Z)) / T.frob(P) < 1e-9


def test_generator_signal_matches_definition():
    w = W.Workload("t", [5, 4, 6, 3], [2, 3, 2, 2], [3, 3, 3, 3], 0, 2, None, 1)
    X, G = W.make_tensor(w)
    np.testing.assert_allclose(X.numpy(), T.tr_full(G), atol=1e-11)


def test_generator_snr():
    w = W.Workload("t", [20, 20, 20, 20], [3] * 4, [8] * 4, 0, 2, 20.0, 2)
    X, G = W.make_tensor(w)
    S = T.tr_full(G)
    snr = 20 * np.log10(T.frob(S) / T.frob(X.numpy() - S))
    assert abs(snr - 20.0) < 0.05


def test_generator_noise_is_the_published_philox_stream():
    """The generator's noise stream is element e of the Philox4x32-10 / Box-Muller stream
    (tag 3), the same definition the oracle's generator is pinned to by the known-answer
    vectors: both the per-element and the four-per-call routes."""
    import torch
    from oracle import philox
    seed, tid = 20190107, 5
    sw = philox.stream_word(3, 0)
    assert sw == W.NOISE_STREAM
    start = (1 << 33) + 3
    ref = philox.normals(seed, sw, tid, start, 1001)
    e = torch.arange(start, start + 1001, dtype=torch.int64)
    np.testing.assert_allclose(W.stream_normals(seed, sw, tid, e).numpy(), ref, rtol=0, atol=1e-15)
    np.testing.assert_allclose(W._stream_run(seed, sw, tid, start, 1001, "cpu").numpy(), ref,
                               rtol=0, atol=1e-15)


def test_generator_block_is_exact_slice_of_full_tensor():
    """A block workload is the leading block of the full tensor: same cores, same sigma,
    noise keyed by the full index (the 64^4 sample of the 200^4 workload, at 12^4 of 40^4)."""
    full = W.dense_200(I=40)
    blk = W.dense_200_block(block=12, I=40)
    Xf, Gf = W.make_tensor(full)
    Xb, Gb = W.make_tensor(blk)
    assert list(Xb.shape) == [12] * 4
    np.testing.assert_allclose(Xb.numpy(), Xf.numpy()[:12, :12, :12, :12], rtol=0,
                               atol=1e-12 * float(np.abs(Xf.numpy()).max()))
    for a, b in zip(Gb, Gf):
        np.testing.assert_array_equal(a, b[:, :12, :])


def test_generator_signal_norm_closed_form():
    G = cores([5, 4, 6, 3], [2, 3, 2, 2], seed=43)
    assert abs(W.tr_norm2(G) - T.frob(T.tr_full(G)) ** 2) < 1e-10 * T.frob(T.tr_full(G)) ** 2
