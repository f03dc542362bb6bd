"""Algorithm 1 (rTRD) of the paper, step by step, in FP64.

Readings of the paper (each applies where the text is silent, ambiguous or garbled):
* Step 4: M is N(0,1) i.i.d.; its entries are the oracle's Philox/Box-Muller stream for
  mode n, element e = j*K_n + k for row j (row-major index of the other-mode multi-index)
  and column k.  Q_n does not depend on the scale of M.
* Step 5: Y_n = X_(n) M is formed from the ORIGINAL tensor X for every mode (M has
  prod_{i!=n} I_i rows), so the N sketches are independent of each other.
* Step 6: economy QR with the sign convention R_ii >= 0 (zero counts as positive).
  K_n >= I_n means mode n is not projected: Q_n is the I_n x I_n identity.
* Step 7 reads cumulatively, as Eq. (3) requires: P = X x_1 Q_1^T x_2 ... x_N Q_N^T.
* Step 9 TR-ALS: initial cores are an input; cores are updated n = 1..N in turn, each by
  the exact least-squares solution of Eq. (2) restricted to P, through the normal equations
  (Cholesky), falling back to minimum-norm least squares if the Gram matrix is not positive
  definite.  Fixed sweep count, or stop once the relative error changes by less than tol.
* Step 11 "Z_n x_n Q_n" on an order-3 core reads as the product over the physical mode
  (mode 2 of the core): G_n = Z_n x_2 Q_n.
* Power iterations (the option named after Alg. 1, Halko et al. 2011 Alg. 4.4): after
  Q = qr(Y), repeat q times W = qr(X_(n)^T Q), Q = qr(X_(n) W).
* RSE (Sec. 4) = ||X - Y||_F / ||X||_F, not squared.

Projection variants (the remark after Alg. 1 names structured test matrices as an option; the
loop of steps 3-8 also admits a sequential reading):
* Khatri-Rao test matrix: M_n is the column-wise Kronecker product of one Gaussian factor
  F_m (I_m x K_n, i.i.d. N(0,1), stream (TAG_KR, mode n, factor m)) per other mode m, rows in
  the column order of X_(n): M_n[j, k] = prod_{m != n} F_m[i_m, k].  It needs sum_{m!=n} I_m
  K_n normals instead of prod_{m!=n} I_m K_n.
* Sequential: the sketch of mode n is taken of the tensor already compressed in modes
  1..n-1, P^(n-1) = X x_1 Q_1^T .. x_{n-1} Q_{n-1}^T (M then has prod_{i<n} K'_i
  prod_{i>n} I_i rows); P is P^(N).
"""
import numpy as np
import scipy.linalg

from . import philox
from .tensor import (unfold, unfold_tr, mode_product, tr_full, subchain, core_fold2,
                     subchain_unfold2, frob)


def gaussian_test_matrix(seed, n, rows, K, tensor_id=0):
    """Alg. 1 step 4: Gaussian M (rows x K) for mode n (0-based).

    Parity: pinned through the Philox known-answer vectors and distribution tests."""
    z = philox.normals(seed, philox.stream_word(philox.TAG_OMEGA, n), tensor_id, 0, rows * K)
    return z.reshape(rows, K)


def khatri_rao_test_matrix(seed, n, dims, K, tensor_id=0):
    """Structured test matrix for mode n (0-based): the Khatri-Rao product of Gaussian factors
    F_m (dims[m] x K) over the other modes m in increasing order, the first of them varying
    slowest (the column order of X_(n)).

    Parity: pinned by the entry-wise definition written as explicit loops over the multi-index,
    by exact range capture for unfoldings of rank <= K, and by its moments."""
    M = np.ones((1, K))
    for m in range(len(dims)):
        if m == n:
            continue
        F = philox.normals(seed, philox.stream_word(philox.TAG_KR, n, m), tensor_id, 0,
                           dims[m] * K).reshape(dims[m], K)
        M = (M[:, None, :] * F[None, :, :]).reshape(-1, K)
    return M


def qr_pos(Y):
    """Alg. 1 step 6: economy QR (Householder, LAPACK) with R_ii >= 0.

    Parity: pinned against the Cholesky route R = chol(Y^T Y), Q = Y R^-1 and orthonormality."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :], R * s[:, None]


def range_basis(X, n, K, q=0, seed=0, tensor_id=0, test="gaussian"):
    """Q_n of Alg. 1 steps 4-6, with q power iterations (Halko et al. 2011, Alg. 4.4).
    ``test`` = "khatri_rao" takes the structured test matrix instead of the Gaussian one.

    Parity: pinned by the exact-arithmetic identity Q = qr((A A^T)^q A M) and the range
    captured for matrices with known singular values."""
    In = X.shape[n]
    if K >= In:
        return np.eye(In)
    A = unfold(X, n)
    if test == "khatri_rao":
        M = khatri_rao_test_matrix(seed, n, X.shape, K, tensor_id)
    else:
        M = gaussian_test_matrix(seed, n, A.shape[1], K, tensor_id)
    Q, _ = qr_pos(A @ M)
    for _ in range(q):
        W, _ = qr_pos(A.T @ Q)
        Q, _ = qr_pos(A @ W)
    return Q


def compress(X, Qs):
    """Alg. 1 step 7 read cumulatively (Eq. 3): P = X x_1 Q_1^T ... x_N Q_N^T.

    Parity: pinned by multilinearity, mode-order independence and the Pythagorean identity."""
    P = X
    for n, Q in enumerate(Qs):
        P = mode_product(P, Q.T, n)
    return P


def sequential_bases(X, K, seed=0, tensor_id=0):
    """Alg. 1 steps 3-8 with step 7 read sequentially: mode n is sketched (Gaussian M of the
    same stream as the independent reading, rows = columns of the current unfolding) from
    P^(n-1), then P^(n) = P^(n-1) x_n Q_n^T.  Returns (Q_1..Q_N, P).

    Parity: pinned by mode 1 equal to the independent reading, by the independent reading
    whenever every earlier mode is kept (K_m >= I_m), and by exact recovery of tensors of low
    multilinear rank."""
    P = np.asarray(X, dtype=np.float64)
    Qs = []
    for n in range(P.ndim):
        In = P.shape[n]
        if K[n] >= In:
            Q = np.eye(In)
        else:
            A = unfold(P, n)
            Q, _ = qr_pos(A @ gaussian_test_matrix(seed, n, A.shape[1], K[n], tensor_id))
        Qs.append(Q)
        P = mode_product(P, Q.T, n)
    return Qs, P


def core_shapes(K, ranks):
    N = len(K)
    return [(ranks[n], K[n], ranks[(n + 1) % N]) for n in range(N)]


def als_update(P, Z, n):
    """One TR-ALS core update (Eq. 2 on P): Z_n <- argmin ||P_<n> - Z_{n,(2)} B^T||_F with
    B = G_{!=n,<2>} built from the other cores.  Returns the new core.

    Parity: pinned by exact recovery, the N=2 Eckart-Young limit and monotone decrease."""
    Ra, In, Rb = Z[n].shape
    B = subchain_unfold2(subchain(Z, n))           # J x (Ra*Rb)
    Pn = unfold_tr(P, n)                            # In x J
    Gm = B.T @ B
    Mm = Pn @ B
    try:
        c = scipy.linalg.cho_factor(Gm, lower=True, check_finite=True)
        W = scipy.linalg.cho_solve(c, Mm.T).T
    except np.linalg.LinAlgError:
        W = np.linalg.lstsq(B, Pn.T, rcond=None)[0].T
    return core_fold2(W, Ra, Rb)


def tr_als(P, Z0, sweeps, tol=0.0, record_updates=False):
    """Alg. 1 step 9 with TR-ALS: ``sweeps`` passes over n = 1..N from the cores Z0.

    After each sweep the relative error ||P - Psi(Z)|| / ||P|| is recorded; with tol > 0 the
    loop stops after sweep s >= 2 once |err(s) - err(s-1)| < tol.
    Returns (cores, per-sweep errors[, per-update errors])."""
    Z = [np.array(z, dtype=np.float64, copy=True) for z in Z0]
    N = len(Z)
    nP = frob(P)
    trace, upd = [], []
    for s in range(sweeps):
        for n in range(N):
            Z[n] = als_update(P, Z, n)
            if record_updates:
                upd.append(frob(P - tr_full(Z)) / nP)
        trace.append(frob(P - tr_full(Z)) / nP)
        if tol > 0 and s >= 1 and abs(trace[-1] - trace[-2]) < tol:
            break
    if record_updates:
        return Z, np.array(trace), np.array(upd)
    return Z, np.array(trace)


def _split_rank(r):
    """R_1 * R_2 = r with R_1 <= R_2 and R_2 - R_1 as small as possible."""
    a = int(np.floor(np.sqrt(r)))
    while r % a:
        a -= 1
    return a, r // a


def _trunc_rank(s, delta):
    """Smallest rank whose discarded singular values have 2-norm <= delta."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])  # tail[r] = ||s[r:]||
    for r in range(1, len(s) + 1):
        if r == len(s) or tail[r] <= delta:
            return r
    return len(s)


def _svd_fixed_sign(C):
    """Economy SVD with a fixed sign per singular pair: each left singular vector is
    negated (with its right partner) unless its entry of largest magnitude (the first such
    on ties) is positive.  TR-SVD needs this because the first rank is split over both
    ends of the ring, which makes the result depend on these signs."""
    U, s, Vt = np.linalg.svd(C, full_matrices=False)
    idx = np.argmax(np.abs(U), axis=0)          # first index of the largest |entry|
    sign = np.where(U[idx, np.arange(U.shape[1])] < 0, -1.0, 1.0)
    return U * sign, s, Vt * sign[:, None]


def tr_svd(P, eps, steps=None):
    """Alg. 1 step 9 with TR-SVD (sequential truncated SVDs, Zhao et al. 2016):
    per-step budget delta = eps ||P|| / sqrt(N), the first step sqrt(2) delta; the first
    rank r_1 is split as R_1 R_2 = r_1 with R_1 <= R_2 as close as possible; the last core
    closes the ring through R_1.  Returns (cores, ranks [R_1..R_N]).  If ``steps`` is a
    list, one (matrix, budget, kept rank) record per truncation is appended to it.

    Parity: pinned by the error bound ||P - Psi(Z)|| <= eps ||P||, by the minimality of every
    truncation (each kept rank is the smallest within its budget, checked on singular values
    obtained by another route), and by the error being exactly the root sum of the discarded
    tails; the exact cores are partly unpinned (the rank split is a reading).  Singular
    vectors follow the sign rule of ``_svd_fixed_sign`` (a reading: the split first rank
    makes the later truncations depend on those signs)."""
    shape = P.shape
    N = len(shape)
    nP = frob(P)
    delta = eps * nP / np.sqrt(N)
    C = P.reshape(shape[0], -1)
    U, s, Vt = _svd_fixed_sign(C)
    r = _trunc_rank(s, np.sqrt(2.0) * delta)
    if steps is not None:
        steps.append((C, np.sqrt(2.0) * delta, r))
    R1, R2 = _split_rank(r)
    Z = [np.transpose(U[:, :r].reshape(shape[0], R1, R2), (1, 0, 2))]
    C = (s[:r, None] * Vt[:r]).reshape(R1, R2, -1)
    C = np.transpose(C, (1, 2, 0))                     # R2 x (K_2..K_N) x R1
    ranks = [R1, R2]
    for k in range(1, N - 1):
        Rk = ranks[-1]
        C = C.reshape(Rk * shape[k], -1)
        U, s, Vt = _svd_fixed_sign(C)
        r = _trunc_rank(s, delta)
        if steps is not None:
            steps.append((C, delta, r))
        Z.append(U[:, :r].reshape(Rk, shape[k], r))
        C = s[:r, None] * Vt[:r]
        ranks.append(r)
    Z.append(C.reshape(ranks[-1], shape[-1], R1))
    return Z, ranks[:N]


def backproject(Z, Qs):
    """Alg. 1 steps 10-12 read as G_n = Z_n x_2 Q_n: G_n[a, i, b] = sum_k Q_n[i, k] Z_n[a, k, b].

    Parity: pinned by multilinearity Psi([Z_n x_2 Q_n]) = Psi([Z_n]) x_1 Q_1 ... x_N Q_N."""
    return [np.einsum("ik,akb->aib", Q, z) for z, Q in zip(Z, Qs)]


def rse(X, G):
    """RSE = ||X - Psi([G_n])||_F / ||X||_F (Sec. 4)."""
    return frob(X - tr_full(G)) / frob(X)


def rtr_als(X, K, Z0, sweeps, q=0, seed=0, tol=0.0, tensor_id=0, projection="gaussian"):
    """The whole of Alg. 1 with TR-ALS.  ``Z0`` are the initial cores of shape
    (R_n, K_n', R_{n+1}) with K_n' = min(K_n, I_n).  ``projection``: "gaussian" (as printed),
    "khatri_rao" (structured test matrices) or "sequential" (step 7 read sequentially, q = 0).
    Returns a dict of every stage."""
    X = np.asarray(X, dtype=np.float64)
    if projection == "sequential":
        assert q == 0
        Qs, P = sequential_bases(X, K, seed, tensor_id)
    else:
        test = "khatri_rao" if projection == "khatri_rao" else "gaussian"
        Qs = [range_basis(X, n, K[n], q, seed, tensor_id, test) for n in range(X.ndim)]
        P = compress(X, Qs)
    Z, trace = tr_als(P, Z0, sweeps, tol)
    G = backproject(Z, Qs)
    return {"Q": Qs, "P": P, "Z": Z, "rse_trace": trace, "G": G, "rse": rse(X, G)}
