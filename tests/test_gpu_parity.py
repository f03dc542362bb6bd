"""GPU parity of every stage of Alg. 1 against the FP64 oracle, through the C ABI.

Tolerances (relative Frobenius differences): FP64 path 1e-10, FP32 path 1e-5, BF16 sketch
path 3e-3.  Q_n is compared directly where Y_n has full column rank (the R_ii >= 0 QR is
then unique); otherwise the projector Q Q^T is compared.
"""
import numpy as np

import conditioning as C
import pytest
import torch

import paper_1901_01652_amd as rt
from paper_1901_01652_amd import pipeline
from oracle import philox as oph, rtr as orc, tensor as ot
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    hd = rt.Handle(0)
    yield hd
    hd.close()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(*a):
    print(*a, flush=True)


def rand_tensor(dims, seed):
    return np.random.default_rng(seed).standard_normal(dims)


def gpu_q(h, X, K, q=0, seed=0, compute=None, tensor_id=0):
    Xd = torch.as_tensor(X).to(DEV)
    Q = rt.rtr_sketch(h, Xd, K, q, seed, tensor_id, compute)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in rt.unpack(Q, rt.q_shapes(X.shape, K))], Q, Xd


# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("start,count", [(0, 1000), (3, 37), (1 << 33, 64), (5, 1)])
def test_normals_match_oracle(h, start, count):
    say("normals", start, count)
    sw = oph.stream_word(oph.TAG_OMEGA, 2)
    ref = oph.normals(12345, sw, 7, start, count)
    g64 = rt.rtr_normals(h, 12345, sw, 7, start, count, "f64").cpu().numpy()
    g32 = rt.rtr_normals(h, 12345, sw, 7, start, count, "f32").cpu().numpy()
    # FP64 Box-Muller: a few ulp (libm and ocml round log/sin/cos independently)
    assert np.max(np.abs(g64 - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-14 or \
        np.max(np.abs(g64 - ref)) < 4 * np.finfo(np.float64).eps * np.max(np.abs(ref))
    # FP32 transcendental unit: small absolute error
    assert np.max(np.abs(g32 - ref)) < 2e-5


@pytest.mark.parametrize("dims,K,q", [
    ((20, 20, 20, 20), (8, 8, 8, 8), 0),
    ((37, 23, 41), (5, 7, 3), 0),
    ((6, 7, 5, 4, 3), (3, 3, 2, 2, 2), 0),
    ((70, 9, 33), (64, 1, 33), 0),          # K = I for the last mode, K = 1, K = 64
    ((30, 20, 25), (6, 5, 4), 1),
    ((30, 20, 25), (6, 5, 4), 2),
    ((150, 70), (12, 10), 1),
])
def test_sketch_fp64(h, dims, K, q):
    say("sketch f64", dims, K, q)
    X = rand_tensor(dims, 1)
    Qg, _, _ = gpu_q(h, X, K, q, seed=99)
    for n in range(len(dims)):
        Qo = orc.range_basis(X, n, K[n], q, seed=99)
        assert rel(Qg[n], Qo) < 1e-10, (n, rel(Qg[n], Qo))
        assert np.max(np.abs(Qg[n].T @ Qg[n] - np.eye(Qg[n].shape[1]))) < 1e-13


# the matrix-core passes pick a loader per mode: cols4 (B % 4 == 0), last4 (last mode,
# I_n % 4 == 0) or scalar; these shapes reach all three, ragged tiles and K = 64.  Tolerance:
# the path's per-stage accuracy times the oracle's own amplification of a relative error in the
# sketch and power products (tests/conditioning.py, sketch_condition).
@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("dims,K,q", [((40, 30, 20, 10), (8, 7, 6, 5), 0),
                                      ((24, 36, 40), (9, 20, 12), 0),
                                      ((13, 7, 9, 11), (5, 3, 4, 6), 0),
                                      ((24, 36, 40), (9, 20, 12), 1),
                                      ((13, 7, 9, 11), (5, 3, 4, 6), 1),
                                      ((200, 12, 16), (40, 6, 8), 1),
                                      # BF16: the last two modes in one slab pass (ragged strips
                                      # and 32-wide chunks, K = 32, K < 16)
                                      ((300, 52, 28), (9, 20, 12), 0),
                                      ((300, 52, 28), (9, 20, 12), 1),
                                      ((17, 19, 36, 44), (5, 6, 20, 32), 1),
                                      ((16, 17, 64, 64), (4, 4, 7, 20), 1),
                                      # modes longer than 256 rows, sketched in row blocks:
                                      # cols4 in 4 x 256, last4 in 176/176/168, scalar in
                                      # 160/141, and K = 60 over 1024 rows
                                      ((1024, 24, 20), (20, 8, 8), 0),
                                      ((12, 40, 520), (6, 8, 30), 0),
                                      ((10, 20, 301), (4, 6, 12), 0),
                                      ((1024, 16, 24), (60, 6, 12), 0)])
def test_sketch_low_precision(h, compute, tol, dims, K, q):
    say("sketch", compute, dims, K, q)
    X = rand_tensor(dims, 2).astype(np.float32)
    Qg, _, _ = gpu_q(h, X, K, q, seed=5, compute=compute)
    probe = C.sketch_condition(X.astype(np.float64), K, q, seed=5)
    for n in range(len(dims)):
        Qo, cp, cq = probe[n]
        ep, eq = rel(Qg[n] @ Qg[n].T, Qo @ Qo.T), rel(Qg[n], Qo)
        say("  mode", n, f"proj {ep:.3g} (limit {tol * max(1, cp):.3g}) Q {eq:.3g} (limit {tol * max(1, cq):.3g})")
        assert ep <= tol * max(1.0, cp), (n, ep, cp)
        assert eq <= tol * max(1.0, cq), (n, eq, cq)
        assert np.max(np.abs(Qg[n].T @ Qg[n] - np.eye(Qg[n].shape[1]))) < 1e-12


@pytest.mark.parametrize("dims,K", [((20, 20, 20, 20), (8, 8, 8, 8)), ((37, 23, 41), (5, 7, 41)),
                                    ((6, 7, 5, 4, 3), (3, 3, 2, 2, 2)), ((9, 11), (4, 11))])
def test_compress_fp64(h, dims, K):
    say("compress f64", dims, K)
    X = rand_tensor(dims, 3)
    Qg, Qd, Xd = gpu_q(h, X, K, 0, seed=4)
    pn2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    P = rt.rtr_compress(h, Xd, K, Qd, p_norm2=pn2).cpu().numpy()
    Po = orc.compress(X, Qg)
    assert rel(P, Po) < 1e-12
    assert abs(pn2.item() - np.sum(Po ** 2)) < 1e-12 * np.sum(Po ** 2)


# shapes for the fused last-two-modes pass: 16-byte and scalar loads, ragged row blocks,
# order 3 and 4, and one below the slab-count threshold (general mode products)
@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
@pytest.mark.parametrize("dims,K", [((33, 20, 17, 12), (8, 7, 6, 5)), ((300, 40, 52), (9, 20, 12)),
                                    ((260, 33, 29), (5, 30, 7)), ((16, 17, 40, 36), (3, 4, 17, 9)),
                                    ((9, 8, 30, 20), (4, 4, 6, 5)),
                                    # BF16: one wavefront per slab (>= 512 slabs): ragged strips
                                    # and chunks, slabs of the dense workload's shape, K = 32
                                    ((600, 30, 44), (9, 20, 12)), ((520, 200, 200), (5, 20, 20)),
                                    ((1024, 16, 28), (4, 16, 7)), ((8, 80, 36, 64), (3, 5, 32, 32))])
def test_compress_low_precision(h, compute, tol, dims, K):
    say("compress", compute, dims, K)
    X = rand_tensor(dims, 6).astype(np.float32)
    Qo = [orc.range_basis(X.astype(np.float64), n, K[n], 0, seed=3) for n in range(len(dims))]
    Qd = rt.pack(Qo, DEV)
    P = rt.rtr_compress(h, torch.as_tensor(X).to(DEV), K, Qd, compute).cpu().numpy()
    Po = orc.compress(X.astype(np.float64), Qo)
    # bf16 operands with the FP32 refinement terms keep P within FP32-class error
    assert rel(P, Po) < (tol / 10 if compute == "bf16" else tol), rel(P, Po)


def als_case(dims, R, seed, noise=0.05):
    G = W.tr_cores(seed, dims, [max(2, r) for r in R])
    P = ot.tr_full(G) + noise * np.random.default_rng(seed).standard_normal(dims) * np.std(ot.tr_full(G))
    Z0 = W.init_cores(seed + 1, dims, R)
    return P, Z0


@pytest.mark.parametrize("dims,R,sweeps", [((8, 8, 8, 8), (3, 3, 3, 3), 10),
                                           ((9, 7, 8), (2, 3, 4), 15),
                                           ((6, 5, 7, 4, 5), (2, 2, 3, 2, 2), 6),
                                           ((20, 15), (2, 3), 10),
                                           ((12, 10, 11), (1, 1, 1), 5),
                                           ((60, 16, 12), (10, 10, 10), 4),
                                           ((70, 9, 8), (3, 4, 3), 4)])
@pytest.mark.parametrize("launch", [0, 1])
def test_als_fp64(h, dims, R, sweeps, launch):
    """launch 0: one cooperative launch for the whole decomposition (ranks <= 6), 1: two
    launches per core update."""
    say("als f64", dims, R, "launch", launch)
    rt.rtr_set_als_launch(h, launch)
    P, Z0 = als_case(dims, R, 11)
    Zo, tro = orc.tr_als(P, Z0, sweeps)
    Z, tr, ns = rt.rtr_decompose(h, torch.as_tensor(P).to(DEV), R, rt.pack(Z0, DEV), sweeps)
    assert rt.rtr_status_sync(h) == 0
    assert int(ns.item()) == sweeps
    Zg = [z.cpu().numpy() for z in rt.unpack(Z, rt.core_shapes(dims, R))]
    rt.rtr_set_als_launch(h, 0)
    assert rel(tr.cpu().numpy(), tro) < 1e-10
    assert rel(ot.tr_full(Zg), ot.tr_full(Zo)) < 1e-10


@pytest.mark.parametrize("launch", [0, 1])
def test_als_tolerance_stop(h, launch):
    dims, R = (7, 6, 8), (2, 2, 2)
    say("als tol", dims, R, "launch", launch)
    rt.rtr_set_als_launch(h, launch)
    P, Z0 = als_case(dims, R, 13, noise=0.3)
    Zo, tro = orc.tr_als(P, Z0, 60, tol=1e-4)
    Z, tr, ns = rt.rtr_decompose(h, torch.as_tensor(P).to(DEV), R, rt.pack(Z0, DEV), 60, tol=1e-4)
    n = int(ns.item())
    rt.rtr_set_als_launch(h, 0)
    assert n == len(tro) and n < 60
    assert rel(tr.cpu().numpy()[:n], tro) < 1e-10
    Zg = [z.cpu().numpy() for z in rt.unpack(Z, rt.core_shapes(dims, R))]
    assert rel(ot.tr_full(Zg), ot.tr_full(Zo)) < 1e-10


@pytest.mark.parametrize("dims,K,R", [((13, 11, 9, 10), (5, 4, 3, 6), (2, 3, 2, 3)),
                                      ((20, 15, 30, 12), (4, 4, 4, 4), (3, 2, 4, 2))])
def test_backproject_and_residual(h, dims, K, R):
    """FP64 residual to 1e-10; FP32 input (Psi on the FP32 matrix cores, sums in FP64) to the
    FP32 path's 1e-5 on the residual.  The second shape spans several 128 x 256 tiles with
    ragged edges on both sides."""
    say("backproject/residual", dims, K, R)
    rng = np.random.default_rng(7)
    Qs = [np.linalg.qr(rng.standard_normal((d, k)))[0] for d, k in zip(dims, K)]
    Z = W.tr_cores(9, K, R)
    G = rt.rtr_backproject(h, dims, K, R, rt.pack(Z, DEV), rt.pack(Qs, DEV))
    Gg = [g.cpu().numpy() for g in rt.unpack(G, rt.core_shapes(dims, R))]
    Go = orc.backproject(Z, Qs)
    for a, b in zip(Gg, Go):
        assert rel(a, b) < 1e-13
    X = ot.tr_full(Go) + 0.1 * rng.standard_normal(dims)
    for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):
        Xd = torch.as_tensor(X).to(dt).to(DEV)
        out = rt.rtr_residual(h, Xd, R, G).cpu().numpy()
        Xh = Xd.double().cpu().numpy()
        assert abs(out[1] - np.sum(Xh ** 2)) < 1e-12 * np.sum(Xh ** 2)
        r2 = ot.frob(Xh - ot.tr_full(Go)) ** 2
        assert abs(out[0] - r2) < tol * r2, (dt, out[0], r2)


def run_end_to_end(h, w, X, compute=None):
    Z0 = W.make_init(w)
    Xd = torch.as_tensor(X).to(DEV)
    out = pipeline.rtr_als(h, Xd, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute, tol=w.tol)
    torch.cuda.synchronize()
    G = [g.cpu().numpy() for g in rt.unpack(out["G"], rt.core_shapes(w.dims, w.ranks))]
    return out, G, pipeline.rse(h, Xd, w.ranks, out["G"]), Z0


def test_end_to_end_small_fp64(h):
    """The 20^4 FP64 workload (rank 3, 40 dB, K=8, 20 sweeps) against the oracle."""
    w = W.small_fp64()
    say("end-to-end", w.name)
    X, _ = W.make_tensor(w)
    X = X.numpy()
    out, G, rse_g, Z0 = run_end_to_end(h, w, X)
    ref = orc.rtr_als(X, w.K, Z0, w.sweeps, q=w.q, seed=w.seed)
    Q = [t.cpu().numpy() for t in rt.unpack(out["Q"], rt.q_shapes(w.dims, w.K))]
    for n in range(4):
        assert rel(Q[n], ref["Q"][n]) < 1e-10
    assert rel(out["P"].cpu().numpy(), ref["P"]) < 1e-10
    assert rel(out["err_trace"].cpu().numpy(), ref["rse_trace"]) < 1e-10
    assert rel(ot.tr_full(G), ot.tr_full(ref["G"])) < 1e-10
    assert abs(rse_g - ref["rse"]) / ref["rse"] < 1e-10
    # Pythagorean identity on the device quantities
    pn2 = out["p_norm2"].item()
    e = out["err_trace"].cpu().numpy()[-1]
    xn2 = float(np.sum(X ** 2))
    rse_py = np.sqrt((xn2 - pn2 + e * e * pn2) / xn2)
    assert abs(rse_py - rse_g) / rse_g < 1e-9


@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 3e-3)])
def test_end_to_end_small_low_precision(h, compute, tol):
    w = W.small_fp64()
    say("end-to-end", w.name, compute)
    X, _ = W.make_tensor(w, dtype=torch.float32)
    X = X.numpy()
    out, G, rse_g, Z0 = run_end_to_end(h, w, X, compute)
    ref = orc.rtr_als(X.astype(np.float64), w.K, Z0, w.sweeps, q=w.q, seed=w.seed)
    assert abs(rse_g - ref["rse"]) / ref["rse"] < tol
    assert rel(ot.tr_full(G), ot.tr_full(ref["G"])) < tol * (30 if compute == "bf16" else 10)


def test_determinism(h):
    w = W.Workload("det", [17, 13, 11, 9], [2, 2, 2, 2], [5, 4, 4, 3], 1, 5, 30.0, 3)
    say("determinism", w.name)
    X, _ = W.make_tensor(w, dtype=torch.float32)
    outs = []
    for _ in range(2):
        out, G, rse_g, _ = run_end_to_end(h, w, X.numpy(), "f32")
        outs.append((out["Q"].cpu(), out["P"].cpu(), out["G"].cpu(), rse_g))
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert torch.equal(a, b)
    assert outs[0][3] == outs[1][3]


def test_invalid_arguments(h):
    say("invalid args")
    X = torch.zeros((4, 5, 6), dtype=torch.float64, device=DEV)
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_sketch(h, X, [0, 2, 2])
    assert e.value.code == 1
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_sketch(h, X, [2, 2, 2], compute="bf16")
    assert e.value.code == 2
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_sketch(h, X, [2, 2, 100])       # K'=I: fine; K>64 on a projected mode is not
        rt.rtr_sketch(h, torch.zeros((4, 5, 100), dtype=torch.float64, device=DEV), [2, 2, 80])
    assert e.value.code == 2
    P = torch.zeros((3, 3, 3), dtype=torch.float64, device=DEV)
    Z0 = torch.zeros(3 * 3 * 5 * 5, dtype=torch.float64, device=DEV)
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose(h, P, [5, 5, 5], Z0, 2)  # R_n R_{n+1} = 25 > 9 equations
    assert e.value.code == 1
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose(h, P, [1, 1, 1], Z0, 2, method="svd")  # ranks are an output
    assert e.value.code == 1


@pytest.mark.parametrize("launch", [0, 1])
def test_cholesky_failure_flag(h, launch):
    """A zero core makes the subchain of the first update vanish, so its Gram matrix is
    exactly zero: the status bit is set, the update skipped, and no kernel faults."""
    dims, R = (5, 6, 7), (2, 2, 2)
    say("cholesky flag", "launch", launch)
    rt.rtr_set_als_launch(h, launch)
    P = torch.as_tensor(rand_tensor(dims, 8)).to(DEV)
    Z0 = [np.ones((2, 5, 2)), np.zeros((2, 6, 2)), np.ones((2, 7, 2))]
    rt.rtr_decompose(h, P, R, rt.pack(Z0, DEV), 1)
    bits = rt.rtr_status_sync(h)
    rt.rtr_set_als_launch(h, 0)
    assert bits & rt.RTR_STATUS_CHOLESKY_FAILED
    assert not bits & rt.RTR_STATUS_SYNC_TIMEOUT
    assert rt.rtr_status_sync(h) == 0
