#!/usr/bin/env python3
"""End-to-end rTR-ALS benchmark on one MI355X (Alg. 1 of arXiv:1901.01652).

Workload: order-4 tensor 200^4 FP32 (6.4 GB) built from random rank-6 TR cores (N(0,1)) plus
30 dB Gaussian noise; projection K=20 per mode with one power iteration; TR-ALS rank 6,
30 sweeps from N(0,1) cores.  One step = sketch + QR + power iteration + compression +
TR-ALS + back-projection, with X resident in HBM when the timed region starts.

Prints one JSON line: end-to-end time per decomposition (ms), the relative error it
reached, the roofline of the dominant X-streaming kernel (HIP events on its launch
stream), the plain-FP32 path beside the BF16 path, and the FP64 oracle timed on the host
cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (scaled by what the counters read for kernels of known traffic), valid only for the kernel
# source they were taken on.
TRAFFIC = {"power_fused": {"bytes_per_launch": 6408565302, "workload": "dense-200^4 bf16",
                           "source": "paper_1901_01652_amd/csrc/fastpass.hip",
                           "sha256": "da0d87f5c111a3dcca1a5aa77c44e52b45aedbf9bfb3bdb60d5f886dacadd4fc",
                           "profile": "profiles/dense200_hbm_traffic_counters.md"}}


def measured_traffic(kernel, workload):
    """Counter-measured bytes per launch, or None if the kernel changed since."""
    import hashlib
    rec = TRAFFIC.get(kernel)
    if not rec or rec["workload"] != workload:
        return None
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["sha256"]:
            return None
    return rec["bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Kernels timed at profiling level 1 (those that stream X), the stage of Alg. 1 each belongs
# to, and how many modes one launch covers (for the per-launch share of the stage's bytes).
KERNEL_STAGE = {"sketch_partial": "sketch", "sketch_fused": "sketch", "sketch_slab": "sketch",
                "power_partial": "power", "power_fused": "power", "power_slab": "power",
                "ttm_first": "compress", "compress_fused": "compress", "sketch_kr_allmode": "sketch"}
MODES_PER_LAUNCH = {"sketch_partial": 1, "sketch_fused": 1, "sketch_slab": 2,
                    "power_partial": 1, "power_fused": 1, "power_slab": 2}


def measure_read_peak(rt, h, X, reps=5):
    """Achievable HBM read rate: the library's 16-byte read-stream probe over X, median of
    ``reps`` launches timed with HIP events on the launch stream."""
    import torch
    rt.rtr_read_probe(h, X)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        rt.rtr_profile_reset(h)
        rt.rtr_profile_enable(h, 1)
        rt.rtr_read_probe(h, X)
        rt.rtr_profile_enable(h, 0)
        ms, n = rt.rtr_profile_read(h, "read_probe")
        times.append(ms / max(n, 1))
    rt.rtr_profile_reset(h)
    ms = float(np.median(times))
    nbytes = X.numel() * X.element_size()
    return {"gbps": round(nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4), "bytes": nbytes}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(I_full, block=64, reps=3):
    """The FP64 oracle, stage by stage, on the leading block^4 block of the dense workload
    (exactly X[:block, ..] of the I_full^4 tensor: same cores, noise and sigma), median of
    ``reps`` runs per stage.  ``value`` scales the stages that stream X (Gaussian draws, sketch
    and power products, compression) by (I_full / block)^4 and the QR by I_full / block; TR-ALS
    and back-projection work on the same K^4 projected tensor and are not scaled."""
    import torch
    from threadpoolctl import threadpool_info
    import workloads as W
    from oracle import rtr as orc
    from oracle.tensor import unfold

    w = W.dense_200_block(block, I=I_full)
    X, _ = W.make_tensor(w, dtype=torch.float32)
    X = X.numpy().astype(np.float64)
    Z0 = W.make_init(w)
    names = ("rng", "sketch_gemm", "qr", "power_gemm", "compress", "tr_als", "backproject")
    runs = {k: [] for k in names}
    pc = time.perf_counter
    for _ in range(reps):
        t = dict.fromkeys(names, 0.0)
        Qs = []
        for n in range(X.ndim):
            t0 = pc()
            A = unfold(X, n)
            t1 = pc()
            M = orc.gaussian_test_matrix(w.seed, n, A.shape[1], w.K[n])
            t2 = pc()
            Y = A @ M
            t3 = pc()
            Q, _ = orc.qr_pos(Y)
            t4 = pc()
            t["sketch_gemm"] += (t1 - t0) + (t3 - t2)
            t["rng"] += t2 - t1
            t["qr"] += t4 - t3
            for _ in range(w.q):
                t0 = pc()
                B = A.T @ Q
                t1 = pc()
                Wq, _ = orc.qr_pos(B)
                t2 = pc()
                Y = A @ Wq
                t3 = pc()
                Q, _ = orc.qr_pos(Y)
                t4 = pc()
                t["power_gemm"] += (t1 - t0) + (t3 - t2)
                t["qr"] += (t2 - t1) + (t4 - t3)
            Qs.append(Q)
        t0 = pc()
        P = orc.compress(X, Qs)
        t1 = pc()
        Z, _ = orc.tr_als(P, Z0, w.sweeps)
        t2 = pc()
        orc.backproject(Z, Qs)
        t3 = pc()
        t["compress"] = t1 - t0
        t["tr_als"] = t2 - t1
        t["backproject"] = t3 - t2
        for k in names:
            runs[k].append(t[k])
    med = {k: float(np.median(v)) for k, v in runs.items()}
    f4 = (I_full / block) ** 4
    f1 = I_full / block
    scaled = {"rng": f4, "sketch_gemm": f4, "power_gemm": f4, "compress": f4, "qr": f1,
              "tr_als": 1.0, "backproject": f1}
    est_s = sum(med[k] * scaled[k] for k in names)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": round(est_s * 1e3, 1), "unit": "ms", "cores": int(threads), "kind": "oracle",
            "sample": (f"FP64 oracle per stage on the {block}^4 block X[:{block}]^4 of the "
                       f"{I_full}^4 tensor (K=20, q=1, rank 6, 30 sweeps), median of {reps}; "
                       f"X-streaming stages scaled by ({I_full}/{block})^4 = {f4:.1f}, QR by "
                       f"{f1:.3g}, TR-ALS unscaled"),
            "block_ms_per_stage": {k: round(v * 1e3, 1) for k, v in med.items()},
            "block_ms": round(sum(med.values()) * 1e3, 1),
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}


def gpu_block(rt, h, I_full, compute, block=64, reps=5):
    """The GPU path on the same block^4 block, for a like-for-like line beside the oracle."""
    import torch
    import workloads as W
    from paper_1901_01652_amd import pipeline
    w = W.dense_200_block(block, I=I_full)
    X, _ = W.make_tensor(w, device="cuda:0", dtype=torch.float32)
    Z0 = rt.pack(W.make_init(w), "cuda:0")
    pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"ms": round(ms, 3), "rse": round(pipeline.rse(h, X, w.ranks, out["G"]), 6),
            "compute": compute}


def bench_hsi(rt, h, steps=5, scale=1):
    """The hyperspectral-shaped workload (1024 x 1024 x 256 FP32 at scale 1, smooth rank-10
    spatial cores, [0, 1], 30 dB; K = (60, 60, 40), q = 0; TR-ALS rank 10, 30 sweeps): time per
    decomposition for the BF16 and plain FP32 paths, each stage's share of the method's
    algorithmic bytes (one read of X for the sketch of all modes, one for the compression),
    and the errors."""
    import torch
    import workloads as W
    from paper_1901_01652_amd import pipeline
    dev = "cuda:0"
    w = W.hsi_shaped(scale=scale)
    log(f"[bench] generating {w.name}")
    X, _ = W.make_tensor(w, device=dev, dtype=torch.float32)
    Z0 = rt.pack(W.make_init(w), dev)
    stream = torch.cuda.current_stream(dev)
    xbytes = w.numel() * 4
    res = {"workload": f"{w.name} fp32, smooth rank-10 spatial cores, [0,1], 30 dB; K={w.K}, q=0; "
                       "TR-ALS rank 10, 30 sweeps", "dims": w.dims, "K": w.K}
    for compute in ("bf16", "f32"):
        pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute)
        torch.cuda.synchronize()
        rt.rtr_profile_reset(h)
        rt.rtr_profile_enable(h, 1)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            out = pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute)
        ev1.record(stream)
        torch.cuda.synchronize()
        rt.rtr_profile_enable(h, 0)
        ms = ev0.elapsed_time(ev1) / steps
        kern, stages = {}, {}
        for name in KERNEL_STAGE:
            tot, n = rt.rtr_profile_read(h, name)
            if n:
                kern[name] = {"avg_ms": round(tot / n, 4), "launches": n}
                st = KERNEL_STAGE[name]
                stages[st] = stages.get(st, 0.0) + tot / steps
        stages = {st: {"ms_per_step": round(v, 4), "alg_bytes": xbytes,
                       "gbps": round(xbytes / (v * 1e-3) / 1e9, 1),
                       "frac": round(xbytes / (v * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
                  for st, v in stages.items()}
        r = rt.rtr_residual(h, X, w.ranks, out["G"]).cpu().numpy()
        nsw = int(out["sweeps_run"].item())
        e = float(out["err_trace"][nsw - 1].item())
        pn2 = float(out["p_norm2"].item())
        res[compute] = {"ms_per_step": round(ms, 3), "rse": round(float(np.sqrt(r[0] / r[1])), 6),
                        "rse_pythagorean": round(float(np.sqrt(max(r[1] - pn2 + e * e * pn2, 0.0) / r[1])), 6),
                        "stages": stages, "kernels": kern}
        log(f"[bench] {w.name} {compute}: {ms:.3f} ms/step, RSE {res[compute]['rse']}")
    del X
    torch.cuda.empty_cache()
    return res


def bench_kr(rt, h, X, w, steps=5):
    """The structured-projection variant on the same tensor: Khatri-Rao test matrices, whose
    BF16 sketch of all modes (and ||X||^2) is one read of X.  Reports the sketch stage alone
    (fraction of the HBM peak for one algorithmic read) and the whole decomposition."""
    import torch
    from paper_1901_01652_amd import pipeline
    stream = torch.cuda.current_stream("cuda:0")
    xbytes = w.numel() * 4
    xn2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    res = {}
    for name, fn in (("sketch", lambda: rt.rtr_sketch(h, X, w.K, 0, w.seed, compute="bf16",
                                                         projection="khatri_rao", x_norm2=xn2)),
                     ("step", lambda: pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed,
                                                       compute="bf16", projection="khatri_rao"))):
        if name == "step":
            import workloads as W
            Z0 = rt.pack(W.make_init(w), "cuda:0")
        fn()
        torch.cuda.synchronize()
        rt.rtr_profile_reset(h)
        rt.rtr_profile_enable(h, 1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        rt.rtr_profile_enable(h, 0)
        ms = e0.elapsed_time(e1) / steps
        tot, n = rt.rtr_profile_read(h, "sketch_kr_allmode")
        res[name] = {"ms": round(ms, 3)}
        if n:
            k_ms = tot / n
            res[name]["one_read_kernel_ms"] = round(k_ms, 4)
            res[name]["one_read_gbps"] = round(xbytes / (k_ms * 1e-3) / 1e9, 1)
            res[name]["one_read_frac"] = round(xbytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        if name == "step":
            res[name]["rse"] = round(pipeline.rse(h, X, w.ranks, out["G"]), 6)
    return res


def _clock(fn, reps=1):
    """Mean wall time (ms) of ``fn`` over ``reps`` calls, the device drained before and after."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps, out


def bench_paper_shapes(rt, h, I=1024, Ks=(50, 75, 100, 125, 150, 175, 200)):
    """Stand-ins for the paper's experiments on synthetic data of their shapes (Sec. 4):

    * Sec. 4.1: a smooth I x I x 3 tensor, projection K x K x 3 over ``Ks`` (from 50: at K = 25
      the first core's least squares has R_1 R_2 = 100 unknowns per row but only K x 3 = 75
      equations), rTR-ALS (rank 10,
      50 sweeps) and rTR-SVD (eps 0.15) against TR-ALS and TR-SVD on the full tensor, on the
      same GPU (TR-SVD on the full tensor at 512 x 512 x 3: its first Gram matrix is I x I and
      the eigen-solver takes at most 512);
    * Sec. 4.2: 32 x 32 x 3 x 50000 and 32 x 32 x 3 x 72 x 100, rTR-SVD and rTR-ALS with time,
      RSE and compression ratio (entries / parameters);
    * Sec. 4.3: 200 x 200 x 80 with K = 100 x 100 x 6 at four noise levels, the RSE against
      the noisy input and against the clean signal.
    Times are wall clock per call with the device drained (BF16 sketch path, FP64 TR-ALS).
    TR-SVD ranks are capped at 32 (the back-projection's rank limit), and in Sec. 4.2 at the
    largest of 32, 16, 8, 4 whose steps keep every Gram within the eigen-solver's 512; "capped"
    reports whether a cap was hit (the eps bound then no longer holds)."""
    import torch
    import workloads as W
    from paper_1901_01652_amd import pipeline
    dev = "cuda:0"
    out = {}

    def params(dims, R):
        N = len(dims)
        return sum(R[n] * dims[n] * R[(n + 1) % N] for n in range(N))

    # --- Sec. 4.1 --------------------------------------------------------------------
    w0 = W.rgb_shaped(I, Ks[0])
    X, _ = W.make_tensor(w0, device=dev, dtype=torch.float32)
    sweep = []
    for K in Ks:
        w = W.rgb_shaped(I, K)
        Z0 = rt.pack(W.make_init(w), dev)
        run = lambda: pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, 0, w.seed, compute="bf16")
        run()
        ms, o = _clock(run)
        rse_als = pipeline.rse(h, X, w.ranks, o["G"])
        runs = lambda: pipeline.rtr_svd(h, X, w.K, [32] * 3, 0.15, 0, w.seed, compute="bf16")
        runs()
        ms_s, os_ = _clock(runs)
        capped = bool(rt.rtr_status_sync(h) & rt.RTR_STATUS_RANK_CAPPED)
        rse_svd = pipeline.rse(h, X, os_["ranks"], os_["G"])
        sweep.append({"K": K, "rtr_als_ms": round(ms, 2), "rtr_als_rse": round(rse_als, 5),
                      "rtr_svd_ms": round(ms_s, 2), "rtr_svd_rse": round(rse_svd, 5),
                      "rtr_svd_ranks": os_["ranks"], "capped": capped})
        log(f"[bench] {w.name}: rTR-ALS {ms:.1f} ms RSE {rse_als:.4f}; rTR-SVD {ms_s:.1f} ms "
            f"RSE {rse_svd:.4f} ranks {os_['ranks']}")
    wf = W.rgb_shaped(I, I)
    Zf = W.init_cores(wf.seed, wf.dims, wf.ranks)
    ms_f, of = _clock(lambda: pipeline.tr_als_full(h, X, wf.ranks, Zf, wf.sweeps))
    rse_f = float(of["err_trace"][int(of["sweeps_run"].item()) - 1])
    log(f"[bench] TR-ALS on the full {I}x{I}x3 tensor: {ms_f:.1f} ms RSE {rse_f:.4f}")
    del X
    # TR-SVD pair at 512 x 512 x 3 (the full tensor's first Gram is 512 x 512)
    w5 = W.rgb_shaped(512, 100)
    X5, _ = W.make_tensor(w5, device=dev, dtype=torch.float32)
    pipeline.rtr_svd(h, X5, w5.K, [32] * 3, 0.15, 0, w5.seed, compute="bf16")
    ms_r5, or5 = _clock(lambda: pipeline.rtr_svd(h, X5, w5.K, [32] * 3, 0.15, 0, w5.seed, compute="bf16"))
    ms_s5, os5 = _clock(lambda: pipeline.tr_svd_full(h, X5, [32] * 3, 0.15))
    svd_pair = {"dims": w5.dims, "K": w5.K,
                "rtr_svd_ms": round(ms_r5, 2), "rtr_svd_rse": round(pipeline.rse(h, X5, or5["ranks"], or5["G"]), 5),
                "rtr_svd_ranks": or5["ranks"], "tr_svd_ms": round(ms_s5, 2),
                "tr_svd_rse": round(float(os5["p_err"].cpu()[0]), 5), "tr_svd_ranks": os5["ranks"]}
    log(f"[bench] 512x512x3: rTR-SVD {ms_r5:.1f} ms, TR-SVD on the full tensor {ms_s5:.1f} ms")
    del X5
    out["sec4_1_simulation"] = {
        "workload": f"smooth {I}x{I}x3 fp32 (rank-12 generator, sigma 8, [0,1], 30 dB); rank 10, "
                    "50 sweeps; eps 0.15", "k_sweep": sweep,
        "tr_als_full": {"ms": round(ms_f, 2), "rse": round(rse_f, 5)}, "tr_svd_pair_512": svd_pair}

    # --- Sec. 4.2 --------------------------------------------------------------------
    coll = []
    for kind in ("cifar", "coil"):
        w = W.images_shaped(kind)
        X, _ = W.make_tensor(w, device=dev, dtype=torch.float32)
        Z0 = rt.pack(W.make_init(w), dev)
        run = lambda: pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, 0, w.seed, compute="bf16")
        run()
        ms, o = _clock(run)
        rse_als = pipeline.rse(h, X, w.ranks, o["G"])
        # the largest uniform rank cap whose TR-SVD steps fit the eigen-solver (at most 512)
        caps = None
        for c in (32, 16, 8, 4):
            try:
                pipeline.rtr_svd(h, X, w.K, [c] * len(w.dims), 0.15, 0, w.seed, compute="bf16")
                caps = [c] * len(w.dims)
                break
            except rt.RtrError as e:
                if e.code != rt.RTR_ERR_UNSUPPORTED:
                    raise
        runs = lambda: pipeline.rtr_svd(h, X, w.K, caps, 0.15, 0, w.seed, compute="bf16")
        ms_s, os_ = _clock(runs)
        capped = bool(rt.rtr_status_sync(h) & rt.RTR_STATUS_RANK_CAPPED)
        rse_svd = pipeline.rse(h, X, os_["ranks"], os_["G"])
        coll.append({"workload": w.name, "K": w.K, "rtr_svd_cap": caps[0], "capped": capped,
                     "rtr_als": {"ranks": w.ranks, "ms": round(ms, 2), "rse": round(rse_als, 5),
                                 "cr": round(w.numel() / params(w.dims, w.ranks), 1)},
                     "rtr_svd": {"ranks": os_["ranks"], "ms": round(ms_s, 2), "rse": round(rse_svd, 5),
                                 "cr": round(w.numel() / params(w.dims, os_["ranks"]), 1)}})
        log(f"[bench] {w.name}: rTR-ALS {ms:.1f} ms RSE {rse_als:.4f}; rTR-SVD {ms_s:.1f} ms "
            f"RSE {rse_svd:.4f} ranks {os_['ranks']}")
        del X, o, os_
    out["sec4_2_compression"] = coll

    # --- Sec. 4.3 --------------------------------------------------------------------
    rec = []
    for snr in (None, 20.0, 10.0, 0.0):
        w = W.hsi_small_shaped(snr)
        clean = []
        X, _ = W.make_tensor(w, device=dev, dtype=torch.float32, clean=clean)
        S = clean[0]
        Z0 = rt.pack(W.make_init(w), dev)
        run = lambda: pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, 0, w.seed, compute="bf16")
        run()
        ms, o = _clock(run)
        rec.append({"snr_db": snr, "ms": round(ms, 2),
                    "rse_vs_input": round(pipeline.rse(h, X, w.ranks, o["G"]), 5),
                    "rse_vs_clean": round(pipeline.rse(h, S, w.ranks, o["G"]), 5)})
        log(f"[bench] {w.name}: {ms:.1f} ms, RSE vs clean {rec[-1]['rse_vs_clean']}")
        del X, S
    out["sec4_3_reconstruction"] = {"workload": "200x200x80 fp32 (rank-10 generator, sigma 2, [0,1]); "
                                                "K=100x100x6, rank 10, 30 sweeps", "runs": rec}
    torch.cuda.empty_cache()
    return out


def bench_tr_svd(rt, h, P, eps=0.15, reps=3):
    """rTR-SVD (Alg. 1 step 9 by TR-SVD) on the projected tensor of the same run."""
    import torch
    caps = [512] * P.dim()
    rt.rtr_decompose_svd(h, P, caps, eps)          # warm-up (workspace, code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Z, ranks, err = rt.rtr_decompose_svd(h, P, caps, eps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"ms": round(ms, 3), "eps": eps, "ranks": [int(r) for r in ranks.cpu()],
            "p_err": round(float(err.cpu()[0]), 6)}


def bench_batched(rt, h, count=512, sweeps=20, reps=3):
    """The batched workload: ``count`` order-4 FP32 tensors with I_n ~ U{16..96},
    R ~ U{2..6}, K = 2R+4, 35 dB, 20 sweeps.  Times the batched pipeline replayed as one HIP
    graph (the work-list form with autotuned tiles and the per-tensor form on 8 branch streams,
    the faster one reported as ``graph_ms``), the same batch run eagerly, and the per-tensor loop
    over the single-tensor calls."""
    import torch
    import workloads as W
    dev = "cuda:0"
    ws = W.batched_uneven(count)
    items = []
    elems = 0
    for w in ws:
        X, _ = W.make_tensor(w, device=dev, dtype=torch.float32)
        items.append({"X": X, "K": list(w.K), "R": list(w.ranks), "Z_init": rt.pack(W.make_init(w), dev),
                      "seed": w.seed, "tensor_id": w.tensor_id})
        elems += X.numel()
    torch.cuda.synchronize()
    log(f"[bench] batched: {count} tensors, {elems / 1e9:.2f} G elements")

    def clock(fn, n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    # tile choice for the work lists (sketch chunks per job, mode-product outputs per thread)
    try:
        table = rt.rtr_batch_autotune(h, items, compute="f32")
    except rt.RtrError as e:
        if e.code != rt.RTR_ERR_UNSUPPORTED:
            raise
        table = None
    # the per-tensor form (8 branch streams in the graph) beside the work lists
    rt.rtr_batch_set_work_lists(h, 0)
    rt.rtr_batch_run(h, items, sweeps, use_graph=True)
    graph_per_tensor_ms = clock(lambda: rt.rtr_batch_run(h, items, sweeps, use_graph=True), reps)
    rt.rtr_batch_set_work_lists(h, 1)
    rt.rtr_batch_run(h, items, sweeps, use_graph=True)      # eager run + graph capture
    graph_lists_ms = clock(lambda: rt.rtr_batch_run(h, items, sweeps, use_graph=True), reps)
    lists = graph_lists_ms <= graph_per_tensor_ms
    rt.rtr_batch_set_work_lists(h, 1 if lists else 0)
    graph_ms = min(graph_lists_ms, graph_per_tensor_ms)
    eager_ms = clock(lambda: rt.rtr_batch_run(h, items, sweeps, use_graph=False), 1)
    rt.rtr_profile_reset(h)
    rt.rtr_profile_enable(h, 2)
    rt.rtr_batch_run(h, items, sweeps, use_graph=False)
    als_ms, _ = rt.rtr_profile_read(h, "als_batch")
    _, sk_launches = rt.rtr_profile_read(h, "sketch_list")
    rt.rtr_batch_set_work_lists(h, 1)
    rt.rtr_profile_enable(h, 0)

    def loop():
        for it in items:
            X = it["X"]
            Q = rt.rtr_sketch(h, X, it["K"], 0, it["seed"], it["tensor_id"], "f32")
            P = rt.rtr_compress(h, X, it["K"], Q, "f32")
            Z, tr, ns = rt.rtr_decompose(h, P, it["R"], it["Z_init"], sweeps)
            rt.rtr_backproject(h, list(X.shape), it["K"], it["R"], Z, Q)

    loop_ms = clock(loop, 1)
    final = [float(it["err_trace"][-1]) for it in items]
    return {"tensors": count, "elements": elems, "graph_ms": round(graph_ms, 2),
            "eager_ms": round(eager_ms, 2), "per_tensor_loop_ms": round(loop_ms, 2),
            "batched_als_kernel_ms": round(als_ms, 2),
            "speedup_vs_loop": round(loop_ms / graph_ms, 2),
            "p_err_median": round(float(np.median(final)), 6), "compute": "f32",
            "sweeps": sweeps, "graph_work_lists_ms": round(graph_lists_ms, 2),
            "graph_per_tensor_ms": round(graph_per_tensor_ms, 2),
            "work_lists_used": sk_launches > 0, "autotune": table}


def bench_warm_start(rt, h, ntrain=2048, max_epochs=80, ntest=32):
    """Learned warm start on the 128^4 rank-4 workload.  The network is trained on the cores
    the method itself reaches (TR-ALS, 30 sweeps, from one fixed set of initial cores) on the
    normalised projected tensors of ``ntrain`` 48^4 inputs of the same recipe (their projected
    tensors have the 12^4 shape of the 128^4 workload's), until the core loss plateaus (mean of
    the last 5 epochs within 1e-3 of the 5 before, at most ``max_epochs``).  Then TR-ALS runs to
    the 1e-4 change criterion from N(0,1) cores and from the prediction on ``ntest`` held-out
    128^4 inputs; the warm arm's time includes the network's inference."""
    import torch
    import workloads as W
    from paper_1901_01652_amd import warmstart as ws
    tpl = W.warm_start_128()
    small = W.warm_start_128(I=48)
    t0 = time.perf_counter()
    data = ws.dataset(h, small, range(1000, 1000 + ntrain))
    Z0 = rt.pack(W.init_cores(small.seed, small.K, small.ranks, 4096), "cuda:0")
    T = ws.method_targets(h, data, small.K, small.ranks, Z0, sweeps=30)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    model = ws.WarmStart(h, tpl.K, tpl.ranks, seed=1)
    t0 = time.perf_counter()
    hist = ws.train_supervised(model, data, T, max_epochs=max_epochs, batch=256, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = ws.evaluate(h, model, tpl, range(ntest))
    arm = lambda k, f: round(float(np.mean([r[k][f] for r in res])), 6)
    return {"train_tensors": ntrain, "train_shape": small.dims, "target": "method cores (30 sweeps)",
            "epochs": len(hist), "train_loss_first": round(hist[0], 5),
            "train_loss_last": round(hist[-1], 5), "dataset_s": round(t_data, 2),
            "train_s": round(t_train, 2), "test_tensors": ntest, "test_shape": tpl.dims,
            "tol": tpl.tol,
            "random": {"sweeps": arm("random", "sweeps"), "p_err": arm("random", "p_err"),
                       "ms": arm("random", "ms")},
            "warm": {"sweeps": arm("warm", "sweeps"), "p_err": arm("warm", "p_err"),
                     "ms": arm("warm", "ms")}}


def bench_sparse(rt, h, dims=(20000, 15000, 10000), nnz=2_000_000, K=(20, 20, 20),
                 R=(4, 4, 4), sweeps=20, reps=3):
    """rTR-ALS of a sparse tensor given by its nonzeros (Sec. 5 names sparse tensors as future
    work): power-law coordinates valued by a rank-4 TR model + 30 dB noise, FP64.  Times per
    call (device drained), the sketch's Gaussian draws per second, and the RSE by the
    Pythagorean identity."""
    import torch
    import workloads as W
    from paper_1901_01652_amd import pipeline
    idx, val, _ = W.sparse_tr(31, dims, list(R), nnz)
    I = torch.as_tensor(idx).to("cuda:0")
    V = torch.as_tensor(val).to("cuda:0")
    Z0 = rt.pack(W.init_cores(31, K, R), "cuda:0")
    xn2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    pipeline.rtr_als_coo(h, I, V, dims, K, R, Z0, sweeps, seed=31)   # warm-up
    ms_sk, Q = _clock(lambda: rt.rtr_sketch_coo(h, I, V, dims, K, seed=31, x_norm2=xn2), reps)
    ms_cp, P = _clock(lambda: rt.rtr_compress_coo(h, I, V, dims, K, Q), reps)
    ms_all, o = _clock(lambda: pipeline.rtr_als_coo(h, I, V, dims, K, R, Z0, sweeps, seed=31), reps)
    x2, p2 = o["x_norm2"].item(), o["p_norm2"].item()
    e = float(o["err_trace"][sweeps - 1])
    rse = float(np.sqrt((x2 - p2 + e * e * p2) / x2))
    normals = nnz * sum(K)
    return {"workload": f"sparse {'x'.join(map(str, dims))}, {nnz} nonzeros (power-law coordinates, "
                        "rank-4 TR values, 30 dB), FP64; K=20, rank 4, 20 sweeps",
            "sketch_ms": round(ms_sk, 3), "compress_ms": round(ms_cp, 3),
            "end_to_end_ms": round(ms_all, 3), "rse": round(rse, 6),
            "sketch_normals_per_s": round(normals / (ms_sk * 1e-3), 1),
            "compress_gflops": round(2.0 * nnz * float(np.prod(K)) / (ms_cp * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--size", type=int, default=200, help="mode size I (default 200)")
    ap.add_argument("--compute", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--no-fp32-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 512-tensor workload")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned warm-start measurement")
    ap.add_argument("--no-tr-svd", action="store_true", help="skip the TR-SVD timing")
    ap.add_argument("--no-hsi", action="store_true",
                    help="skip the hyperspectral-shaped 1024x1024x256 workload")
    ap.add_argument("--no-kr", action="store_true",
                    help="skip the Khatri-Rao projection variant on the dense tensor")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the stand-ins for the paper's experiments (Sec. 4)")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the sparse (coordinate-list) workload")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_1901_01652_amd as rt
    from paper_1901_01652_amd import pipeline
    import workloads as W

    dev = "cuda:0"
    w = W.dense_200(I=args.size)
    log(f"[bench] generating {w.name} on {dev}")
    X, _ = W.make_tensor(w, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    Z0 = rt.pack(W.make_init(w), dev)
    h = rt.Handle(0)
    stream = torch.cuda.current_stream(dev)

    def step(compute):
        return pipeline.rtr_als(h, X, w.K, w.ranks, Z0, w.sweeps, w.q, w.seed, compute=compute)

    def timed(compute, steps, warmup, profile):
        for i in range(warmup):
            step(compute)
        torch.cuda.synchronize()
        rt.rtr_profile_reset(h)
        rt.rtr_profile_enable(h, 1 if profile else 0)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for i in range(steps):
            out = step(compute)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        ms = ev0.elapsed_time(ev1) / steps
        rt.rtr_profile_enable(h, 0)
        return out, ms, wall

    if args.copy_probe:
        # counter calibration: the read-stream probe reads exactly X's bytes (once per call);
        # the Gaussian stream kernel writes exactly 1 GiB of FP32 values and reads nothing
        wbuf = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        rt.rtr_normals(h, 1, 1 << 24, 0, 0, 1 << 28, "f32", out=wbuf)
        torch.cuda.synchronize()
        log("[bench] calibration probes: read_probe_kernel reads X once (6.4e9 B); "
            "normals_kernel writes 1 GiB")
        del wbuf

    read_peak = measure_read_peak(rt, h, X)
    log(f"[bench] read-stream probe over X: {read_peak['gbps']} GB/s")
    log(f"[bench] {args.compute}: warmup {args.warmup}, {args.steps} timed steps")
    out, ms, wall = timed(args.compute, args.steps, args.warmup, True)
    log(f"[bench] {args.compute}: {ms:.2f} ms/step (host wall {wall:.2f})")

    numel = w.numel()
    xbytes = numel * 4
    N = len(w.dims)
    kern = {}
    for name in KERNEL_STAGE:
        tot, n = rt.rtr_profile_read(h, name)
        if n:
            kern[name] = {"total_ms": tot, "launches": n, "avg_ms": tot / n,
                          "stage": KERNEL_STAGE[name],
                          # per-launch HBM efficiency: bytes this launch streams (one read of X)
                          "launch_gbps": round(xbytes / (tot / n * 1e-3) / 1e9, 1)}
    # algorithmic bytes of each stage per step (one read of X for the sketch of every mode,
    # ceil(N/2) reads per power round, one read for the compression) over the stage's
    # measured kernel time per step
    stage_alg = {"sketch": xbytes, "power": w.q * ((N + 1) // 2) * xbytes, "compress": xbytes}
    stages = {}
    for st, alg in stage_alg.items():
        ms_st = sum(k["total_ms"] for k in kern.values() if k["stage"] == st) / args.steps
        if ms_st > 0:
            gbps = alg / (ms_st * 1e-3) / 1e9
            stages[st] = {"alg_bytes": alg, "ms_per_step": round(ms_st, 4), "gbps": round(gbps, 1),
                          "frac": round(gbps / HBM_PEAK_GBPS, 4),
                          "frac_measured_peak": round(gbps / read_peak["gbps"], 4)}
    # dominant kernel; its algorithmic bytes per launch are its stage's bytes per mode times
    # the modes one launch covers
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    st = KERNEL_STAGE[dom]
    alg_launch = stage_alg[st] * MODES_PER_LAUNCH.get(dom, N) / N
    achieved = alg_launch / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(dom, f"dense-{args.size}^4 {args.compute}"),
            "alg_bytes_per_launch": int(alg_launch), "avg_launch_ms": round(kern[dom]["avg_ms"], 4),
            "measured_read_peak_gbps": read_peak["gbps"],
            "frac_measured_peak": round(achieved / read_peak["gbps"], 4)}

    rt.rtr_residual(h, X, w.ranks, out["G"])            # warm-up (workspace)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    res_d = rt.rtr_residual(h, X, w.ranks, out["G"])
    e1.record(stream)
    torch.cuda.synchronize()
    res_ms = e0.elapsed_time(e1)
    res = res_d.cpu().numpy()
    rse = float(np.sqrt(res[0] / res[1]))
    nsw = int(out["sweeps_run"].item())
    e = float(out["err_trace"][nsw - 1].item())
    pn2 = float(out["p_norm2"].item())
    rse_py = float(np.sqrt(max(res[1] - pn2 + e * e * pn2, 0.0) / res[1]))

    kr = None
    if not args.no_kr:
        log("[bench] Khatri-Rao test matrices (one read of X for every mode's sketch)")
        kr = bench_kr(rt, h, X, w)

    fp32 = None
    if not args.no_fp32_compare and args.compute != "f32":
        log("[bench] plain FP32 path for comparison")
        o32, ms32, _ = timed("f32", max(1, args.steps // 2), 1, False)
        r32 = rt.rtr_residual(h, X, w.ranks, o32["G"]).cpu().numpy()
        fp32 = {"ms_per_step": round(ms32, 3), "rse": float(np.sqrt(r32[0] / r32[1]))}

    svd = None
    if not args.no_tr_svd:
        log("[bench] TR-SVD on the projected tensor")
        svd = bench_tr_svd(rt, h, out["P"])
    hsi = None
    if not args.no_hsi:
        hsi = bench_hsi(rt, h)
    paper = None
    if not args.no_paper_shapes:
        paper = bench_paper_shapes(rt, h)
    sparse = None
    if not args.no_sparse:
        log("[bench] sparse tensor, coordinate list")
        sparse = bench_sparse(rt, h)
        log(f"[bench] sparse: sketch {sparse['sketch_ms']} ms, compress {sparse['compress_ms']} ms, "
            f"end to end {sparse['end_to_end_ms']} ms, RSE {sparse['rse']}")
    batched = None
    if not args.no_batched:
        del out
        torch.cuda.empty_cache()
        batched = bench_batched(rt, h)
        log(f"[bench] batched: graph {batched['graph_ms']} ms, loop {batched['per_tensor_loop_ms']} ms")

    warm = None
    if not args.no_warm_start:
        log("[bench] learned warm start (128^4, rank 4)")
        warm = bench_warm_start(rt, h)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] FP64 oracle on the host (bounded sample)")
        cpu = cpu_baseline(args.size)
        cpu["gpu_same_block"] = gpu_block(rt, h, args.size, args.compute)

    line = {
        "metric": "end-to-end rTR-ALS time + sketch HBM GB/s (% roofline) at stated rel. error",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": args.compute, "data": "synthetic",
        "config": {"workload": f"dense order-4 {args.size}^4 fp32 from rank-6 TR cores + 30 dB noise; "
                               "K=20 per mode, 1 power iteration; TR-ALS rank 6, 30 sweeps",
                   "dims": w.dims, "K": w.K, "ranks": w.ranks, "power_iters": w.q,
                   "sweeps": w.sweeps, "compute": args.compute,
                   "fp64": "QR, power-step orthonormalisation, TR-ALS"},
        "rse": round(rse, 6), "rse_pythagorean": round(rse_py, 6), "p_err": round(e, 6),
        "rse_explicit": {"ms": round(res_ms, 3), "gbps": round(xbytes / (res_ms * 1e-3) / 1e9, 1),
                         "note": "one extra pass over X (timed apart from the step)"},
        "roofline": roof, "stages": stages, "read_peak": read_peak, "kernels": kern,
        "fp32_path": fp32, "cpu_baseline": cpu,
        "tr_svd": svd, "khatri_rao": kr, "hsi_shaped": hsi, "paper_shapes": paper, "batched": batched,
        "warm_start": warm, "sparse": sparse,
    }
    h.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
