"""Batched TR-ALS (one persistent launch for many tensors) and the batched Alg. 1 pipeline
(optionally replayed as one HIP graph), against the FP64 oracle, through the C ABI.

Tolerances: FP64 path 1e-10 on the per-sweep error trace (relative), 1e-9 on Psi(Z).  FP32
path, stage by stage: P against the oracle's P at 1e-5 (relative Frobenius); the batched TR-ALS
against the oracle's TR-ALS on the GPU's own P at 1e-10 (ALS from a random start can pass
through sensitive transients, so FP32-class differences in P are not compared through it);
Psi(G) against the oracle's back-projection of the GPU's own cores at 1e-5.  The batch with
FP32 X and no power iterations runs its sketches, QRs and mode products as work lists.
"""
import numpy as np
import pytest
import torch

import conditioning as C
import paper_1901_01652_amd as rt
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
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def low_rank_plus_noise(dims, R, noise, rng):
    N = len(dims)
    cores = [rng.standard_normal((R[n], dims[n], R[(n + 1) % N])) for n in range(N)]
    S = ot.tr_full(cores)
    E = rng.standard_normal(dims)
    return S + noise * np.linalg.norm(S) / np.linalg.norm(E) * E


CASES = [
    ((8, 9, 7, 6), (2, 3, 2, 2)),
    ((6, 5, 7), (3, 2, 4)),
    ((12, 10, 11, 9), (6, 6, 6, 6)),
    ((20, 30), (2, 3)),
    ((5, 4, 6, 3, 4), (2, 2, 2, 2, 2)),
    ((16, 16, 16, 16), (6, 6, 6, 6)),
    ((64, 5, 6), (2, 2, 2)),
    ((3, 4, 3), (1, 2, 1)),
]


def make_items(seed, tol_sweeps=6):
    rng = np.random.default_rng(seed)
    items, ref = [], []
    for dims, R in CASES:
        P = low_rank_plus_noise(dims, [max(1, r - 1) for r in R], 0.05, rng)
        Z0 = [rng.standard_normal((R[n], dims[n], R[(n + 1) % len(dims)])) for n in range(len(dims))]
        items.append({"P": torch.as_tensor(P).to(DEV), "R": list(R), "Z_init": rt.pack(Z0, DEV)})
        ref.append((P, Z0, dims, R))
    return items, ref


def test_batched_als_matches_oracle(h):
    say("batched als vs oracle")
    sweeps = 6
    items, ref = make_items(41)
    rt.rtr_decompose_batch(h, items, sweeps)
    assert rt.rtr_status_sync(h) == 0
    for it, (P, Z0, dims, R) in zip(items, ref):
        Zo, trace = orc.tr_als(P, Z0, sweeps)
        g_trace = it["err_trace"].cpu().numpy()
        assert int(it["sweeps_run"].cpu()[0]) == sweeps
        assert np.max(np.abs(g_trace - trace) / np.asarray(trace)) < 1e-10, (dims, g_trace, trace)
        Zg = [z.cpu().numpy() for z in rt.unpack(it["Z"], rt.core_shapes(dims, R))]
        assert rel(ot.tr_full(Zg), ot.tr_full(Zo)) < 1e-9, dims


def test_batched_als_tolerance_stop(h):
    say("batched als tol")
    items, ref = make_items(43)
    tol = 1e-3
    rt.rtr_decompose_batch(h, items, 30, tol=tol)
    for it, (P, Z0, dims, R) in zip(items, ref):
        _, trace = orc.tr_als(P, Z0, 30, tol=tol)
        assert int(it["sweeps_run"].cpu()[0]) == len(trace), dims
        got = it["err_trace"].cpu().numpy()[:len(trace)]
        assert np.max(np.abs(got - trace) / np.asarray(trace)) < 1e-10


def test_batched_als_alias_and_single_item(h):
    """Z may alias Z_init; a batch of one tensor works like any other."""
    say("batched als alias")
    items, ref = make_items(47)
    it = items[2]
    it["Z"] = it["Z_init"]
    rt.rtr_decompose_batch(h, [it], 3)
    P, Z0, dims, R = ref[2]
    Zo, trace = orc.tr_als(P, Z0, 3)
    assert np.max(np.abs(it["err_trace"].cpu().numpy() - trace) / np.asarray(trace)) < 1e-10


def test_batched_als_invalid(h):
    items, _ = make_items(49)
    bad = dict(items[0])
    bad["R"] = [7, 2, 2, 2]
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose_batch(h, [bad], 2)
    assert e.value.code == 2
    bad = dict(items[7])
    bad["R"] = [4, 4, 3]   # R_1 R_2 = 16 > 4 * 3 equations for core 1
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_decompose_batch(h, [bad], 2)
    assert e.value.code == 1


def pipeline_items(count, dtype, lo=10, hi=24):
    ws = W.batched_uneven(count, lo=lo, hi=hi)
    items, ref = [], []
    for w in ws:
        X, _ = W.make_tensor(w)
        Z0 = W.make_init(w)
        items.append({"X": X.to(dtype).to(DEV), "K": list(w.K), "R": list(w.ranks),
                      "Z_init": rt.pack(Z0, DEV), "seed": w.seed, "tensor_id": w.tensor_id})
        ref.append((X.to(dtype).double().numpy(), w, Z0))
    return items, ref


@pytest.mark.parametrize("dtype,tol_trace,tol_psi", [(torch.float64, 1e-10, 1e-9),
                                                    (torch.float32, 1e-5, 1e-5)])
def test_batch_pipeline_matches_oracle(h, dtype, tol_trace, tol_psi):
    """64 seeded order-4 tensors with uneven shapes and ranks (the batched workload's
    distribution, smaller modes so the oracle finishes quickly)."""
    say("batch pipeline", dtype)
    sweeps = 20
    items, ref = pipeline_items(64, dtype)
    rt.rtr_batch_run(h, items, sweeps)
    assert rt.rtr_status_sync(h) == 0
    worst_t = worst_p = 0.0
    rng = np.random.default_rng(5)
    for it, (X, w, Z0) in zip(items, ref):
        o = orc.rtr_als(X, w.K, Z0, sweeps, q=0, seed=w.seed, tensor_id=w.tensor_id)
        g_trace = it["err_trace"].cpu().numpy()
        diff = np.abs(g_trace - o["rse_trace"])
        Pg = it["P"].cpu().numpy()
        assert rel(Pg, o["P"]) < (1e-10 if dtype == torch.float64 else 1e-5)
        if dtype == torch.float64:
            diff = diff / np.asarray(o["rse_trace"])
        else:
            # FP32: P carries FP32-class error, to which TR-ALS from a random start can be
            # sensitive; the batched TR-ALS is held stage-wise, against the oracle's TR-ALS on
            # the GPU's own P
            _, tro = orc.tr_als(Pg, Z0, sweeps)
            diff = np.abs(g_trace - np.asarray(tro)) / np.asarray(tro) * tol_trace / 1e-10
        worst_t = max(worst_t, np.max(diff))
        G = [g.cpu().numpy() for g in rt.unpack(it["G"], rt.core_shapes(w.dims, w.ranks))]
        if dtype == torch.float64:
            worst_p = max(worst_p, rel(ot.tr_full(G), ot.tr_full(o["G"])))
        else:  # Psi(G) of the GPU's cores against the oracle's back-projection of the same cores
            Zg = [z.cpu().numpy() for z in rt.unpack(it["Z"], rt.core_shapes(w.K, w.ranks))]
            Qg = [q.cpu().numpy() for q in rt.unpack(it["Q"], rt.q_shapes(w.dims, w.K))]
            worst_p = max(worst_p, rel(ot.tr_full(G), ot.tr_full(orc.backproject(Zg, Qg))))
    say("worst trace", worst_t, "worst psi(G)", worst_p)
    assert worst_p < tol_psi
    assert worst_t < tol_trace


@pytest.mark.parametrize("count", [16, 3, 1])
def test_batch_graph_replay(h, count):
    """The captured graph replays the whole batch: every replay (with other work and
    synchronisations in between) reproduces the eager outputs bit for bit.  16 tensors fill
    all branch streams of the capture (two per branch, each branch on its own workspace
    slice), 3 leave branches unused, 1 captures a single chain."""
    say("batch graph replay", count)
    items, _ = pipeline_items(count, torch.float32)
    rt.rtr_batch_run(h, items, 10, use_graph=True)       # eager run + capture
    torch.cuda.synchronize()
    want = {k: [it[k].clone() for it in items] for k in ("Q", "P", "Z", "G", "err_trace")}
    for rep in range(3):
        for it in items:
            for k in ("Q", "P", "Z", "G", "err_trace"):
                it[k].fill_(float("nan"))
        junk = torch.randn(1 << 20, device=DEV).sum()       # unrelated eager work
        torch.cuda.synchronize()
        rt.rtr_batch_run(h, items, 10, use_graph=True)   # replay
        torch.cuda.synchronize()
        for k, ref in want.items():
            for it, r in zip(items, ref):
                assert torch.equal(it[k], r), (rep, k)
        del junk


def test_batch_work_lists_real_distribution(h):
    """64 tensors of the batched workload's own distribution (order 4, I_n ~ U{16..96},
    R ~ U{2..6}, K = 2R + 4, 35 dB), FP32: the sketches, QRs and mode products of the whole
    batch as work lists (a few launches), stage by stage against the oracle: every projector at
    the FP32 stage accuracy times the oracle's amplification, P against the oracle's compression
    with the returned bases, and the TR-ALS error trace against the oracle's TR-ALS on the
    returned P (1e-10)."""
    say("batch work lists, I_n in [16, 96]")
    sweeps = 20
    ws = W.batched_uneven(64)
    items, ref = [], []
    for w in ws:
        X, _ = W.make_tensor(w, dtype=torch.float32)
        Z0 = W.make_init(w)
        items.append({"X": X.to(DEV), "K": list(w.K), "R": list(w.ranks), "Z_init": rt.pack(Z0, DEV),
                      "seed": w.seed, "tensor_id": w.tensor_id})
        ref.append((w, Z0))
    rt.rtr_profile_reset(h)
    rt.rtr_profile_enable(h, 2)
    rt.rtr_batch_run(h, items, sweeps, compute="f32")
    torch.cuda.synchronize()
    rt.rtr_profile_enable(h, 0)
    _, nsk = rt.rtr_profile_read(h, "sketch_list")
    assert nsk == 1, "the batch's sketches run as one work-list launch"
    assert rt.rtr_status_sync(h) == 0
    worst = {"proj": 0.0, "P": 0.0, "trace": 0.0}
    for it, (w, Z0) in zip(items, ref):
        X = it["X"].cpu().numpy().astype(np.float64)
        Qg = [q.cpu().numpy() for q in rt.unpack(it["Q"], rt.q_shapes(w.dims, w.K))]
        probe = C.sketch_condition(X, w.K, 0, seed=w.seed, tensor_id=w.tensor_id, samples=2)
        for n in range(4):
            Qo, cp, _ = probe[n]
            e = rel(Qg[n] @ Qg[n].T, Qo @ Qo.T)
            worst["proj"] = max(worst["proj"], e / max(1.0, cp))
            assert e <= 1e-5 * max(1.0, cp), (w.tensor_id, n, e, cp)
        Pg = it["P"].cpu().numpy()
        eP = rel(Pg, orc.compress(X, Qg))
        worst["P"] = max(worst["P"], eP)
        assert eP < 1e-5, (w.tensor_id, eP)
        _, tro = orc.tr_als(Pg, Z0, sweeps)
        et = rel(it["err_trace"].cpu().numpy(), tro)
        worst["trace"] = max(worst["trace"], et)
        assert et < 1e-10, (w.tensor_id, et)
    say("worst", worst)


def test_batch_autotune(h):
    """The autotuner times its candidates on a batch, keeps the fastest pair, and the batch run
    with the chosen tiles gives the same P to FP32 accuracy (the partial sums are taken in
    another order) and, on that P, exactly the oracle's TR-ALS (1e-10): the TR-ALS error trace
    itself is not compared between the two runs, since ALS amplifies the FP32-level change of P
    by the conditioning of these small random problems."""
    say("batch autotune")
    items, ref = pipeline_items(16, torch.float32, lo=16, hi=48)
    rt.rtr_batch_run(h, items, 10, compute="f32")
    before = [(it["P"].cpu().clone(), it["err_trace"].cpu().clone()) for it in items]
    table = rt.rtr_batch_autotune(h, items, compute="f32")
    say("table", table)
    assert table["sketch_chunks_per_job"] in (16, 64, 256)
    assert table["ttm_outputs_per_thread"] in (4, 16, 64)
    assert all(v > 0 for v in table["sketch_us"].values()) and all(v > 0 for v in table["ttm_us"].values())
    rt.rtr_batch_run(h, items, 10, compute="f32")
    for it, (P0, t0), (_, w, Z0) in zip(items, before, ref):
        Pg = it["P"].cpu().numpy()
        assert rel(Pg, P0.numpy()) < 1e-5
        _, tro = orc.tr_als(Pg, Z0, 10)
        assert rel(it["err_trace"].cpu().numpy(), tro) < 1e-10
