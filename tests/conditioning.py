"""Conditioning probe of Alg. 1 on the FP64 oracle: how much each compared quantity moves when
every stage that a GPU pass computes is off by a given relative amount.

The parity tolerances of the plan (FP64 path 1e-10, FP32 path 1e-5, BF16-sketch path 3e-3) are
read as the relative accuracy of each stage's result: the sketch Y_n = X_(n) M_n (Alg. 1 step 5),
each power-iteration product X_(n) W (the option named after Alg. 1), and the projected tensor P
(step 7, Eq. 3).  What that accuracy allows downstream depends on the conditioning of the steps
that follow (QR, TR-ALS from a fixed start), which no fixed factor captures.  The probe measures
it: rerun the oracle's own steps with each of those stage outputs perturbed by a random matrix of
relative Frobenius size ``delta`` and record, per quantity q, the amplification
cond_q = rel_change(q) / delta (largest over a few random directions).  A GPU result then matches
when rel(q_gpu, q_oracle) <= tol * max(1, cond_q).  This is the sensitivity pin of the parity plan
(perturb, rerun the oracle, let the growth factor bound what parity can reach), applied at every
stage instead of only to P.

Test infrastructure: it composes the oracle's step functions (it adds no arithmetic of the
method) and is used only by the tests.
"""
import numpy as np

from oracle import rtr as orc
from oracle.tensor import unfold, tr_full


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def perturbed_rtr_als(X, K, Z0, sweeps, q, seed, delta, rng, tensor_id=0):
    """Alg. 1 by the oracle's steps with Y_n, every power product and P perturbed by a random
    relative ``delta``.  With delta = 0 it is ``oracle.rtr.rtr_als`` step for step."""
    def pert(A):
        if delta == 0.0:
            return A
        E = rng.standard_normal(A.shape)
        return A + (delta * np.linalg.norm(A) / np.linalg.norm(E)) * E

    X = np.asarray(X, dtype=np.float64)
    Qs = []
    for n in range(X.ndim):
        In = X.shape[n]
        if K[n] >= In:
            Qs.append(np.eye(In))
            continue
        A = unfold(X, n)
        M = orc.gaussian_test_matrix(seed, n, A.shape[1], K[n], tensor_id)
        Q, _ = orc.qr_pos(pert(A @ M))
        for _ in range(q):
            W, _ = orc.qr_pos(A.T @ Q)
            Q, _ = orc.qr_pos(pert(A @ W))
        Qs.append(Q)
    P = pert(orc.compress(X, Qs))
    Z, trace = orc.tr_als(P, Z0, sweeps)
    G = orc.backproject(Z, Qs)
    return {"Q": Qs, "P": P, "Z": Z, "rse_trace": trace, "G": G, "rse": orc.rse(X, G)}


def quantities(res):
    """The compared quantities of one run: projectors Q_n Q_n^T, P, the per-sweep error on P,
    Psi(G) and the final RSE."""
    return {"proj": [Q @ Q.T for Q in res["Q"]], "P": res["P"], "trace": res["rse_trace"],
            "psi": tr_full(res["G"]), "rse": res["rse"]}


def distance(a, b, key):
    """Relative difference of quantity ``key`` (largest over modes for the projectors)."""
    if key == "proj":
        return max(rel(x, y) for x, y in zip(a, b))
    if key == "rse":
        return abs(a - b) / abs(b)
    return rel(a, b)


KEYS = ("proj", "P", "trace", "psi", "rse")


def condition(X, K, Z0, sweeps, q, seed, delta=1e-8, samples=2, tensor_id=0):
    """(oracle result, its quantities, cond) with cond[key] the largest amplification over
    ``samples`` random perturbation directions of relative size ``delta``."""
    base = orc.rtr_als(X, K, Z0, sweeps, q=q, seed=seed, tensor_id=tensor_id)
    qb = quantities(base)
    cond = {k: 0.0 for k in KEYS}
    for s in range(samples):
        rng = np.random.default_rng(8191 + s)
        qp = quantities(perturbed_rtr_als(X, K, Z0, sweeps, q, seed, delta, rng, tensor_id))
        for k in KEYS:
            cond[k] = max(cond[k], distance(qp[k], qb[k], k) / delta)
    return base, qb, cond


def sketch_condition(X, K, q, seed, delta=1e-8, samples=6, tensor_id=0, test="gaussian"):
    """Per mode: (oracle basis Q_n, amplification of the projector Q_n Q_n^T, amplification of
    Q_n) when the sketch and every power product of that mode are off by a relative ``delta``.

    The amplification is a maximum over perturbation directions.  Random directions (the
    largest over ``samples``) approach it from below; for the last product Y (K columns) the
    first-order bounds close it from above: the projector moves by at most
    sqrt(2) ||dY|| / sigma_min(Y), i.e. relative amplification sqrt(2) ||Y||_F /
    (sigma_min(Y) sqrt(K)), and the R_ii >= 0 QR factor by at most (1 + sqrt(2)) ||dY|| /
    sigma_min(Y).  Each reported amplification is the larger of the two.  Modes with
    K_n >= I_n report 0."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    for n in range(X.ndim):
        In = X.shape[n]
        if K[n] >= In:
            out.append((np.eye(In), 0.0, 0.0))
            continue
        A = unfold(X, n)
        if test == "khatri_rao":
            M = orc.khatri_rao_test_matrix(seed, n, X.shape, K[n], tensor_id)
        else:
            M = orc.gaussian_test_matrix(seed, n, A.shape[1], K[n], tensor_id)

        last = {}

        def basis(rng):
            def pert(B):
                if rng is None:
                    last["Y"] = B
                    return B
                E = rng.standard_normal(B.shape)
                return B + (delta * np.linalg.norm(B) / np.linalg.norm(E)) * E
            Q, _ = orc.qr_pos(pert(A @ M))
            for _ in range(q):
                W, _ = orc.qr_pos(A.T @ Q)
                Q, _ = orc.qr_pos(pert(A @ W))
            return Q

        Q0 = basis(None)
        Y = last["Y"]
        smin = np.linalg.svd(Y, compute_uv=False)[-1]
        ratio = np.linalg.norm(Y) / (smin * np.sqrt(K[n]))
        cp, cq = np.sqrt(2.0) * ratio, (1.0 + np.sqrt(2.0)) * ratio
        for s in range(samples):
            Qp = basis(np.random.default_rng(4099 + s))
            cp = max(cp, rel(Qp @ Qp.T, Q0 @ Q0.T) / delta)
            cq = max(cq, rel(Qp, Q0) / delta)
        out.append((Q0, cp, cq))
    return out
