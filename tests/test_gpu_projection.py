"""Projection variants through the C ABI against the oracle: Khatri-Rao structured test
matrices (rtr_sketch_kr) and the sequential reading of Alg. 1 step 7 (rtr_sketch_sequential).

FP64 at 1e-10.  FP32 / BF16 sketches at the path's stage accuracy times the oracle's own
amplification of a relative error in the sketch (tests/conditioning.py), as for the Gaussian
sketch.  The sequential variant's later modes are sketched from the FP64 intermediate, so past
the first mode the comparison is stage-wise: each Q_n against the oracle's step applied to the
GPU's own intermediate.
"""
import numpy as np
import pytest
import torch

import conditioning as C
import paper_1901_01652_amd as rt
from paper_1901_01652_amd import pipeline
from oracle import rtr as orc, tensor as ot
from oracle.tensor import unfold, mode_product
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


def qs(Q, dims, K):
    return [t.cpu().numpy() for t in rt.unpack(Q, rt.q_shapes(dims, K))]


@pytest.mark.parametrize("dims,K,q", [((20, 20, 20, 20), (8, 8, 8, 8), 0),
                                      ((20, 20, 20, 20), (8, 8, 8, 8), 1),
                                      ((37, 23, 41), (5, 7, 3), 0),
                                      ((6, 7, 5, 4, 3), (3, 3, 2, 2, 2), 0)])
def test_kr_sketch_fp64(h, dims, K, q):
    say("kr f64", dims, K, q)
    X = np.random.default_rng(41).standard_normal(dims)
    Q = rt.rtr_sketch(h, torch.as_tensor(X).to(DEV), K, q, seed=7, projection="khatri_rao")
    Qg = qs(Q, dims, K)
    for n in range(len(dims)):
        Qo = orc.range_basis(X, n, K[n], q, seed=7, test="khatri_rao")
        assert rel(Qg[n], Qo) < 1e-10, (n, rel(Qg[n], Qo))


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("dims,K,q", [((40, 30, 20, 10), (8, 7, 6, 5), 0),
                                      ((300, 52, 28), (9, 20, 12), 1),    # row blocks, power
                                      ((1024, 24, 20), (20, 8, 8), 0),
                                      ((200, 30, 12), (100, 20, 6), 0),   # column blocks
                                      ((13, 7, 9, 11), (5, 3, 4, 6), 0)])  # scalar loader
def test_kr_sketch_low_precision(h, compute, tol, dims, K, q):
    say("kr", compute, dims, K, q)
    X = np.random.default_rng(42).standard_normal(dims).astype(np.float32)
    Q = rt.rtr_sketch(h, torch.as_tensor(X).to(DEV), K, q, seed=8, compute=compute,
                      projection="khatri_rao")
    Qg = qs(Q, dims, K)
    probe = C.sketch_condition(X.astype(np.float64), K, q, seed=8, test="khatri_rao")
    for n in range(len(dims)):
        Qo, cp, cq = probe[n]
        ep, eq = rel(Qg[n] @ Qg[n].T, Qo @ Qo.T), rel(Qg[n], Qo)
        say("  mode", n, f"proj {ep:.3g} (limit {tol * max(1, cp):.3g}) Q {eq:.3g}")
        assert ep <= tol * max(1.0, cp), (n, ep, cp)
        assert eq <= tol * max(1.0, cq), (n, eq, cq)


def test_kr_end_to_end_small_fp64(h):
    """The 20^4 FP64 workload with Khatri-Rao test matrices, through TR-ALS and back-projection."""
    w = W.small_fp64()
    say("kr end-to-end", w.name)
    X, _ = W.make_tensor(w)
    X = X.numpy()
    Z0 = W.make_init(w)
    out = pipeline.rtr_als(h, torch.as_tensor(X).to(DEV), w.K, w.ranks, Z0, w.sweeps, 0, w.seed,
                           projection="khatri_rao")
    ref = orc.rtr_als(X, w.K, Z0, w.sweeps, seed=w.seed, projection="khatri_rao")
    assert rel(out["P"].cpu().numpy(), ref["P"]) < 1e-10
    assert rel(out["err_trace"].cpu().numpy(), ref["rse_trace"]) < 1e-10
    G = [g.cpu().numpy() for g in rt.unpack(out["G"], rt.core_shapes(w.dims, w.ranks))]
    assert rel(ot.tr_full(G), ot.tr_full(ref["G"])) < 1e-10


@pytest.mark.parametrize("dims,K", [((20, 20, 20, 20), (8, 8, 8, 8)),
                                    ((37, 23, 41), (5, 7, 41)),       # last mode kept
                                    ((30, 20, 25), (30, 5, 4)),       # first mode kept
                                    ((6, 7, 5, 4, 3), (3, 3, 2, 2, 2))])
def test_sequential_fp64(h, dims, K):
    say("sequential f64", dims, K)
    X = np.random.default_rng(43).standard_normal(dims)
    pn2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    Q, P = rt.rtr_sketch_sequential(h, torch.as_tensor(X).to(DEV), K, seed=12, p_norm2=pn2)
    Qo, Po = orc.sequential_bases(X, K, seed=12)
    Qg = qs(Q, dims, K)
    for n in range(len(dims)):
        assert rel(Qg[n], Qo[n]) < 1e-10, (n, rel(Qg[n], Qo[n]))
    assert rel(P.cpu().numpy(), Po) < 1e-10
    assert abs(pn2.item() - np.sum(Po ** 2)) < 1e-10 * np.sum(Po ** 2)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("dims,K", [((40, 30, 20, 10), (8, 7, 6, 5)),
                                    ((300, 52, 28), (100, 20, 12))])   # row and column blocks
def test_sequential_low_precision(h, compute, tol, dims, K):
    say("sequential", compute, dims, K)
    X = np.random.default_rng(44).standard_normal(dims).astype(np.float32)
    Xo = X.astype(np.float64)
    Q, P = rt.rtr_sketch_sequential(h, torch.as_tensor(X).to(DEV), K, seed=13, compute=compute)
    Qg = qs(Q, dims, K)
    # the first mode sees X itself: the plain sketch's comparison
    Qo, cp, cq = C.sketch_condition(Xo, K, 0, seed=13)[0]
    assert rel(Qg[0] @ Qg[0].T, Qo @ Qo.T) <= tol * max(1.0, cp)
    # later modes: the oracle's step on the GPU's own bases (FP64 sketches of the intermediate)
    T = Xo
    for n in range(len(dims)):
        if n > 0:
            A = unfold(T, n)
            Qn, _ = orc.qr_pos(A @ orc.gaussian_test_matrix(13, n, A.shape[1], K[n]))
            assert rel(Qg[n] @ Qg[n].T, Qn @ Qn.T) < tol * 10, (n, rel(Qg[n] @ Qg[n].T, Qn @ Qn.T))
        T = mode_product(T, Qg[n].T, n)
    # P is the product of X with the returned bases, at the path's compression accuracy
    assert rel(P.cpu().numpy(), T) < (tol / 10 if compute == "bf16" else tol)


@pytest.mark.parametrize("dims,K", [((20, 16, 36, 44), (5, 6, 20, 32)),     # order 4, K = 32
                                    ((300, 52, 28), (9, 20, 12)),           # order 3
                                    ((1024, 24, 20), (20, 8, 8)),           # 1024-row mode
                                    ((8, 7, 6, 24, 20), (3, 3, 2, 10, 8)),  # order 5
                                    ((4, 70, 36, 40), (4, 9, 12, 10))])     # first mode kept
def test_kr_one_read_all_modes(h, dims, K):
    """BF16 Khatri-Rao sketch of every mode from one read of X (the slab-streaming kernel, seen
    in the launch profile), with ||X||^2 from the same pass."""
    say("kr one read", dims, K)
    X = np.random.default_rng(45).standard_normal(dims).astype(np.float32)
    xn2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    rt.rtr_profile_reset(h)
    rt.rtr_profile_enable(h, 1)
    Q = rt.rtr_sketch(h, torch.as_tensor(X).to(DEV), K, 0, seed=11, compute="bf16",
                      projection="khatri_rao", x_norm2=xn2)
    torch.cuda.synchronize()
    rt.rtr_profile_enable(h, 0)
    _, launches = rt.rtr_profile_read(h, "sketch_kr_allmode")
    assert launches == 1
    assert abs(xn2.item() - np.sum(X.astype(np.float64) ** 2)) < 1e-6 * np.sum(X.astype(np.float64) ** 2)
    Qg = qs(Q, dims, K)
    probe = C.sketch_condition(X.astype(np.float64), K, 0, seed=11, test="khatri_rao")
    for n in range(len(dims)):
        Qo, cp, cq = probe[n]
        ep = rel(Qg[n] @ Qg[n].T, Qo @ Qo.T)
        say("  mode", n, f"proj {ep:.3g} (limit {3e-3 * max(1, cp):.3g})")
        assert ep <= 3e-3 * max(1.0, cp), (n, ep, cp)
        assert rel(Qg[n], Qo) <= 3e-3 * max(1.0, cq)
