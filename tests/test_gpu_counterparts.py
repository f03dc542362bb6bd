"""Wide projections and the traditional counterparts, through the C ABI, against the oracle.

* Projection sizes above 64 (the sketch and the power step in column blocks of at most 64,
  mode products with K up to 256), with the conditioning-scaled tolerance of the other sketch
  tests (tests/conditioning.py).
* TR-ALS with K'_n up to 1024 and R_n R_{n+1} up to 100 (outputs of the accumulation split into
  blocks over the grid), at 1e-10 against the oracle's TR-ALS.
* The counterparts the paper compares against (Sec. 4.1): TR-ALS and TR-SVD on the full tensor.
  With K_n = I_n the randomized method reduces to them exactly (every Q_n is the identity), so
  the full-tensor calls are held to the oracle's plain TR-ALS / TR-SVD at 1e-10, and rTR-ALS
  with K = I to the same numbers.
* rTR-SVD end to end (sketch, compression, TR-SVD, back-projection) against the oracle.
"""
import numpy as np
import pytest
import torch

import conditioning as C
import paper_1901_01652_amd as rt
from paper_1901_01652_amd import pipeline
from oracle import rtr as orc, tensor as ot
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    hd = rt.Handle(0)
    yield hd
    hd.close()


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("dims,K,q", [((200, 30, 12), (100, 20, 6), 0),   # 64 + 36 columns
                                      ((200, 30, 12), (100, 20, 6), 1),   # power step in blocks
                                      ((200, 12, 16), (64, 6, 8), 1),     # FP32 power: 2 x 32
                                      ((150, 40, 36), (130, 10, 8), 0),   # 64 + 64 + 2
                                      ((1024, 6, 24), (150, 4, 8), 0)])   # row x column blocks
def test_sketch_wide(h, compute, tol, dims, K, q):
    say("wide sketch", compute, dims, K, q)
    X = np.random.default_rng(7).standard_normal(dims).astype(np.float32)
    Xd = torch.as_tensor(X).to(DEV)
    Q = rt.rtr_sketch(h, Xd, K, q, seed=17, compute=compute)
    torch.cuda.synchronize()
    Qg = [t.cpu().numpy() for t in rt.unpack(Q, rt.q_shapes(dims, K))]
    probe = C.sketch_condition(X.astype(np.float64), K, q, seed=17)
    for n in range(len(dims)):
        Qo, cp, cq = probe[n]
        ep, eq = rel(Qg[n] @ Qg[n].T, Qo @ Qo.T), rel(Qg[n], Qo)
        say("  mode", n, f"proj {ep:.3g} (limit {tol * max(1, cp):.3g}) Q {eq:.3g}")
        assert ep <= tol * max(1.0, cp), (n, ep, cp)
        assert eq <= tol * max(1.0, cq), (n, eq, cq)


@pytest.mark.parametrize("compute,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_compress_wide(h, compute, tol):
    dims, K = (200, 30, 12), (100, 20, 6)
    say("wide compress", compute, dims, K)
    X = np.random.default_rng(8).standard_normal(dims)
    if compute == "f32":
        X = X.astype(np.float32)
    Qo = [orc.range_basis(X.astype(np.float64), n, K[n], 0, seed=3) for n in range(3)]
    P = rt.rtr_compress(h, torch.as_tensor(X).to(DEV), K, rt.pack(Qo, DEV),
                        None if compute == "f64" else compute).cpu().numpy()
    assert rel(P, orc.compress(X.astype(np.float64), Qo)) < tol


def als_case(dims, R, seed, noise=0.05):
    G = W.tr_cores(seed, dims, R)
    S = ot.tr_full(G)
    P = S + noise * np.random.default_rng(seed).standard_normal(dims) * np.std(S)
    return P, W.init_cores(seed + 1, dims, R)


@pytest.mark.parametrize("dims,R,sweeps", [((100, 12, 10), (10, 10, 10), 4),   # 20000 outputs
                                           ((300, 20, 8), (8, 8, 8), 4),        # K'_1 = 300
                                           ((1024, 12, 3), (3, 3, 3), 4)])      # K'_1 = 1024
def test_als_wide(h, dims, R, sweeps):
    say("wide als", dims, R)
    P, Z0 = als_case(dims, R, 31)
    Zo, tro = orc.tr_als(P, Z0, sweeps)
    Z, tr, ns = rt.rtr_decompose(h, torch.as_tensor(P).to(DEV), R, rt.pack(Z0, DEV), sweeps)
    assert rt.rtr_status_sync(h) == 0
    Zg = [z.cpu().numpy() for z in rt.unpack(Z, rt.core_shapes(dims, R))]
    say("  trace", rel(tr.cpu().numpy(), tro), "psi", rel(ot.tr_full(Zg), ot.tr_full(Zo)))
    assert rel(tr.cpu().numpy(), tro) < 1e-10
    assert rel(ot.tr_full(Zg), ot.tr_full(Zo)) < 1e-10


def test_full_tr_als_is_the_counterpart(h):
    """TR-ALS on the full 20^4 FP64 workload tensor (rank 3, 20 sweeps) equals the oracle's
    plain TR-ALS on X, and rTR-ALS with K = I equals it too."""
    w = W.small_fp64()
    say("full TR-ALS", w.name)
    X, _ = W.make_tensor(w)
    X = X.numpy()
    Z0 = W.init_cores(w.seed, w.dims, w.ranks)
    Zo, tro = orc.tr_als(X, Z0, w.sweeps)
    Xd = torch.as_tensor(X).to(DEV)
    full = pipeline.tr_als_full(h, Xd, w.ranks, Z0, w.sweeps)
    Zg = [z.cpu().numpy() for z in rt.unpack(full["Z"], rt.core_shapes(w.dims, w.ranks))]
    assert rel(full["err_trace"].cpu().numpy(), tro) < 1e-10
    assert rel(ot.tr_full(Zg), ot.tr_full(Zo)) < 1e-10
    # the per-sweep error of TR-ALS on X is the RSE of Sec. 4
    assert abs(tro[-1] - orc.rse(X, Zo)) < 1e-12
    rand = pipeline.rtr_als(h, Xd, w.dims, w.ranks, Z0, w.sweeps)
    Gg = [g.cpu().numpy() for g in rt.unpack(rand["G"], rt.core_shapes(w.dims, w.ranks))]
    assert rel(ot.tr_full(Gg), ot.tr_full(Zo)) < 1e-10


@pytest.mark.parametrize("eps", [0.15, 0.05])
def test_full_tr_svd_is_the_counterpart(h, eps):
    w = W.small_fp64()
    say("full TR-SVD", w.name, eps)
    X, _ = W.make_tensor(w)
    X = X.numpy()
    caps = [64] * 4
    full = pipeline.tr_svd_full(h, torch.as_tensor(X).to(DEV), caps, eps)
    Zo, ranks_o = orc.tr_svd(X, eps)
    assert rt.rtr_status_sync(h) == 0
    assert full["ranks"] == list(ranks_o)
    cores = [c.cpu().numpy() for c in rt.svd_cores(full["Z"], full["ranks"], w.dims, caps)]
    assert rel(ot.tr_full(cores), ot.tr_full(Zo)) < 1e-10


@pytest.mark.parametrize("compute,tol", [(None, 1e-10), ("f32", 1e-5)])
def test_rtr_svd_end_to_end(h, compute, tol):
    """rTR-SVD (eps 0.15) on a 40^3 rank-3 tensor with K = 20 (chosen ranks 3, 3, 20): ranks
    exactly, Psi(G) against the oracle's sketch + compression + TR-SVD + back-projection."""
    dims, K, eps = (40, 40, 40), (20, 20, 20), 0.15
    rng = np.random.default_rng(5)
    cores = [rng.standard_normal((3, d, 3)) for d in dims]
    S = ot.tr_full(cores)
    X = S + 0.001 * np.linalg.norm(S) / np.sqrt(S.size) * rng.standard_normal(dims)
    if compute == "f32":
        X = X.astype(np.float32)
    Xo = X.astype(np.float64)
    Qs = [orc.range_basis(Xo, n, K[n], 0, seed=9) for n in range(3)]
    Zo, ranks_o = orc.tr_svd(orc.compress(Xo, Qs), eps)
    Go = orc.backproject(Zo, Qs)
    out = pipeline.rtr_svd(h, torch.as_tensor(X).to(DEV), K, [64] * 3, eps, seed=9, compute=compute)
    assert rt.rtr_status_sync(h) == 0
    assert out["ranks"] == list(ranks_o)
    G = [g.cpu().numpy() for g in rt.unpack(out["G"], rt.core_shapes(dims, out["ranks"]))]
    assert rel(ot.tr_full(G), ot.tr_full(Go)) < tol
