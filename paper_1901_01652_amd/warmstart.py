"""Learned warm start for TR-ALS, driven through the C ABI (``rtr_mlp_*``).

A multilayer perceptron maps the normalised projected tensor P~ = P / ||P|| to the packed
initial cores of Alg. 1 step 9; it is trained on ||P~ - Psi(Z)||^2 over projected tensors
that the method itself produced (sketch + compression of synthetic inputs), and its
prediction, scaled by ||P||^(1/N) per core, replaces the N(0,1) initial cores.

This module only orchestrates: every product, the loss, its gradient, the optimiser step
and the conversions run in the library's kernels.
"""
import numpy as np
import torch

from . import (rtr_compress, rtr_decompose, rtr_mlp_adam, rtr_mlp_backward, rtr_mlp_core_loss,
               rtr_mlp_forward, rtr_mlp_normalize, rtr_mlp_to_cores, rtr_mlp_tr_loss, rtr_sketch,
               core_shapes, pack)


class WarmStart:
    """The network and its Adam state (FP32 master weights on the device)."""

    def __init__(self, h, K, R, hidden=(1024, 1024, 1024), seed=0, device="cuda:0",
                 compute="bf16"):
        self.h, self.K, self.R, self.compute = h, list(K), list(R), compute
        d_in = int(np.prod(K))
        d_out = sum(a * b * c for a, b, c in core_shapes(K, R))
        self.sizes = [d_in, *hidden, d_out]
        g = torch.Generator(device="cpu").manual_seed(int(seed))
        self.W, self.b = [], []
        for a, c in zip(self.sizes[:-1], self.sizes[1:]):
            # He initialisation; the output layer starts small so Psi(Z) starts near zero
            std = (2.0 / a) ** 0.5 if c != d_out else 0.1 / a ** 0.5
            self.W.append((torch.randn((a, c), generator=g) * std).to(device))
            self.b.append(torch.zeros(c, device=device))
        # output bias: N(0,1) cores scaled by (prod K * prod R)^(-1/(2N)), so that Psi of them
        # has norm ~1 (each entry of Psi of N(0,1) cores has variance prod R); a nonzero start
        # keeps the gradient through the product of the other cores away from zero
        N = len(K)
        c = (float(np.prod(K)) * float(np.prod(R))) ** (-1.0 / (2 * N))
        self.b[-1].copy_((torch.randn(d_out, generator=g) * c).to(device))
        self.m = [torch.zeros_like(t) for t in self.W + self.b]
        self.v = [torch.zeros_like(t) for t in self.W + self.b]
        self.step = 0

    def forward(self, x):
        return rtr_mlp_forward(self.h, self.W, self.b, x, compute=self.compute)

    def train_step(self, x, lr=1e-3):
        """One Adam step on a batch of normalised tensors x (B x prod K); returns the mean
        loss as a device scalar."""
        y, acts = self.forward(x)
        loss, dy = rtr_mlp_tr_loss(self.h, y, x, self.K, self.R, 1.0 / x.shape[0])
        dW, db = rtr_mlp_backward(self.h, self.W, x, acts, dy, compute=self.compute)
        self.step += 1
        for p, gr, m, v in zip(self.W + self.b, dW + db, self.m, self.v):
            rtr_mlp_adam(self.h, p, gr, m, v, self.step, lr)
        return loss.mean()

    def train_step_supervised(self, x, t, lr=1e-3):
        """One Adam step on the supervised core loss against targets t (B x packed cores)."""
        y, acts = self.forward(x)
        loss, dy = rtr_mlp_core_loss(self.h, y, t, 1.0 / x.shape[0])
        dW, db = rtr_mlp_backward(self.h, self.W, x, acts, dy, compute=self.compute)
        self.step += 1
        for p, gr, m, v in zip(self.W + self.b, dW + db, self.m, self.v):
            rtr_mlp_adam(self.h, p, gr, m, v, self.step, lr)
        return loss.mean()

    def init_cores(self, P, p_norm2):
        """Packed FP64 initial cores for projected tensors P (B x K_1..K_N, FP64) with
        ||P||^2 in p_norm2 (B, device)."""
        B = P.shape[0]
        x = rtr_mlp_normalize(self.h, P.reshape(B, -1))
        y, _ = self.forward(x)
        return rtr_mlp_to_cores(self.h, y, p_norm2, order=len(self.K))


def projected(h, w, compute="bf16"):
    """Alg. 1 steps 3-7 for workload ``w`` on the device: (X, Q, P, ||P||^2)."""
    from workloads import make_tensor
    X, _ = make_tensor(w, device="cuda:0", dtype=torch.float32)
    Q = rtr_sketch(h, X, w.K, w.q, w.seed, w.tensor_id, compute)
    pn2 = torch.zeros(1, dtype=torch.float64, device=X.device)
    P = rtr_compress(h, X, w.K, Q, compute, p_norm2=pn2)
    return X, Q, P, pn2


def dataset(h, template, ids, compute="bf16"):
    """Normalised projected tensors (len(ids) x prod K, FP32) of the workload ``template``
    with tensor ids ``ids`` (seeded inputs; training and test ids are kept disjoint)."""
    import dataclasses
    K = template.K
    out = torch.empty((len(ids), int(np.prod(K))), dtype=torch.float32, device="cuda:0")
    for r, t in enumerate(ids):
        w = dataclasses.replace(template, tensor_id=int(t))
        X, Q, P, _ = projected(h, w, compute)
        rtr_mlp_normalize(h, P.reshape(1, -1), out=out[r:r + 1])
        del X
    return out


def evaluate(h, model, template, ids, max_sweeps=100, tol=1e-4, compute="bf16"):
    """For each test tensor: TR-ALS from the N(0,1) initial cores and from the warm start
    (stop once the error changes by less than tol).  Returns per-tensor dicts with the sweeps
    run, the final error on P and the TR-ALS (+ warm-start inference) time in ms."""
    import dataclasses
    from workloads import make_init
    out = []
    for t in ids:
        w = dataclasses.replace(template, tensor_id=int(t))
        X, Q, P, pn2 = projected(h, w, compute)
        del X
        rec = {"tensor_id": int(t)}
        Zr = pack(make_init(w), P.device)  # the random start is given, not timed
        for arm in ("random", "warm"):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            ev0.record()
            if arm == "random":
                Z0 = Zr
            else:
                Z0 = model.init_cores(P.unsqueeze(0), pn2).reshape(-1)
            Z, trace, nsw = rtr_decompose(h, P, w.ranks, Z0, max_sweeps, tol)
            ev1.record()
            torch.cuda.synchronize()
            ns = int(nsw.item())
            rec[arm] = {"sweeps": ns, "p_err": float(trace[ns - 1]), "ms": ev0.elapsed_time(ev1)}
        out.append(rec)
    return out


def train(model, data, epochs, batch=256, lr=1e-3, seed=0, log=None):
    """Mini-batch Adam over ``data``; returns the mean loss of every epoch."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    n = data.shape[0]
    hist = []
    for ep in range(epochs):
        order = torch.randperm(n, generator=g).to(data.device)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            x = data.index_select(0, order[s:s + batch]).contiguous()
            tot += float(model.train_step(x, lr))
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"[warm-start] epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def train_until(model, data, max_epochs=200, batch=256, lr=1e-3, window=5, rel_tol=1e-3,
                seed=0, log=None):
    """Mini-batch Adam until the loss plateaus: stop once the mean loss of the last ``window``
    epochs differs from that of the ``window`` before by less than ``rel_tol`` (relative), or
    after ``max_epochs``.  Returns the per-epoch mean losses."""
    hist = []
    for ep in range(max_epochs):
        hist += train(model, data, 1, batch, lr, seed + ep)
        if log:
            log(f"[warm-start] epoch {ep}: loss {hist[-1]:.6f}")
        if len(hist) >= 2 * window:
            a = sum(hist[-window:]) / window
            b = sum(hist[-2 * window:-window]) / window
            if abs(a - b) <= rel_tol * abs(b):
                break
    return hist


def method_targets(h, data, K, R, Z0, sweeps=30):
    """Cores the method itself produces for each normalised projected tensor (rows of ``data``):
    TR-ALS from the one fixed set of initial cores ``Z0`` (packed, device), so that every
    target is in the gauge that ALS reaches from the same start.  Returns B x packed FP32."""
    B = data.shape[0]
    out = torch.empty((B, Z0.numel()), dtype=torch.float32, device=data.device)
    for r in range(B):
        P = data[r].reshape(list(K)).to(torch.float64)
        Z, _, _ = rtr_decompose(h, P, R, Z0, sweeps)
        out[r].copy_(Z)
    return out


def train_supervised(model, data, targets, max_epochs=200, batch=256, lr=1e-3, window=5,
                     rel_tol=1e-3, seed=0, log=None):
    """Mini-batch Adam on the supervised core loss until it plateaus (as ``train_until``)."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    n = data.shape[0]
    hist = []
    for ep in range(max_epochs):
        order = torch.randperm(n, generator=g).to(data.device)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = order[s:s + batch]
            x = data.index_select(0, idx).contiguous()
            t = targets.index_select(0, idx).contiguous()
            tot += float(model.train_step_supervised(x, t, lr))
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"[warm-start] epoch {ep}: core loss {hist[-1]:.6f}")
        if len(hist) >= 2 * window:
            a = sum(hist[-window:]) / window
            b = sum(hist[-2 * window:-window]) / window
            if abs(a - b) <= rel_tol * abs(b):
                break
    return hist
