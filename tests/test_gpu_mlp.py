"""Warm-start MLP kernels (forward, TR loss and its gradient, backward, Adam) against the
FP64 oracle, through the C ABI.

Tolerances (relative Frobenius): FP32 products 1e-5 on activations and the loss, 1e-4 on
gradients (sums over the batch and the long input dimension in FP32); bf16 products 2e-2
(both operands rounded to 8 significant bits, FP32 accumulation).
"""
import numpy as np
import pytest
import torch

import paper_1901_01652_amd as rt
from oracle import mlp as om

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
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def net(sizes, seed):
    """He-scaled weights, small biases (FP32 values, the oracle sees the same numbers)."""
    rng = np.random.default_rng(seed)
    W = [(rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32)
         for a, b in zip(sizes[:-1], sizes[1:])]
    b = [(0.01 * rng.standard_normal(n)).astype(np.float32) for n in sizes[1:]]
    return W, b


def to_dev(arrs):
    return [torch.as_tensor(a).to(DEV) for a in arrs]


def inputs(B, dims, seed):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((B, int(np.prod(dims))))
    x = (P / np.linalg.norm(P, axis=1, keepdims=True)).astype(np.float32)
    return P, x


SMALL_K, SMALL_R = (3, 4, 2, 3), (2, 3, 2, 2)
SMALL_OUT = sum(a * b * c for a, b, c in om.core_shapes(SMALL_K, SMALL_R))
C5_K, C5_R = (12, 12, 12, 12), (4, 4, 4, 4)


def test_normalize(h):
    P = torch.as_tensor(np.random.default_rng(1).standard_normal((3, 500))).to(DEV)
    out = rt.rtr_mlp_normalize(h, P).cpu().numpy()
    ref = P.cpu().numpy()
    ref = ref / np.linalg.norm(ref, axis=1, keepdims=True)
    assert np.max(np.abs(out - ref)) < 1e-7


@pytest.mark.parametrize("sizes,B", [([72, 64, 48, SMALL_OUT], 5),
                                     ([20736, 1024, 1024, 1024, 768], 4)])
@pytest.mark.parametrize("compute,tol", [("f32", 1e-5), ("bf16", 2e-2)])
def test_forward_matches_oracle(h, sizes, B, compute, tol):
    say("mlp forward", sizes, compute)
    W, b = net(sizes, 2)
    dims = SMALL_K if sizes[0] == 72 else C5_K
    _, x = inputs(B, dims, 3)
    y, acts = rt.rtr_mlp_forward(h, to_dev(W), to_dev(b), torch.as_tensor(x).to(DEV),
                                 compute=compute)
    yo, acts_o = om.forward([(w.astype(np.float64), c.astype(np.float64)) for w, c in zip(W, b)],
                            x.astype(np.float64))
    assert rel(y.cpu().numpy(), yo) < tol
    for a, ao in zip(acts, acts_o[1:]):
        assert rel(a.cpu().numpy(), ao) < tol


@pytest.mark.parametrize("K,R", [(SMALL_K, SMALL_R), (C5_K, C5_R)])
def test_tr_loss_and_core_gradient(h, K, R):
    say("mlp tr loss", K, R)
    B = 3
    dout = sum(a * b * c for a, b, c in om.core_shapes(K, R))
    rng = np.random.default_rng(4)
    y = (0.5 * rng.standard_normal((B, dout))).astype(np.float32)
    _, tgt = inputs(B, K, 5)
    scale = 1.0 / B
    loss, dy = rt.rtr_mlp_tr_loss(h, torch.as_tensor(y).to(DEV), torch.as_tensor(tgt).to(DEV),
                                  K, R, scale)
    psi = om.psi_batch(y.astype(np.float64), K, R)
    D = psi - tgt
    assert rel(loss.cpu().numpy(), np.sum(D * D, axis=1)) < 1e-5
    ref = np.stack([np.concatenate([g.reshape(-1) for g in om._psi_grad_cores(
        om.unpack_cores(y[s].astype(np.float64), K, R), (2.0 * scale * D[s]).reshape(K))])
        for s in range(B)])
    assert rel(dy.cpu().numpy(), ref) < 1e-5


def test_backward_matches_oracle(h):
    """Forward, TR loss and backward on the GPU (FP32 products) against the oracle's
    gradients of the mean loss."""
    say("mlp backward")
    sizes = [72, 64, 48, SMALL_OUT]
    B = 6
    W, b = net(sizes, 6)
    P, x = inputs(B, SMALL_K, 7)
    Wd, bd, xd = to_dev(W), to_dev(b), torch.as_tensor(x).to(DEV)
    y, acts = rt.rtr_mlp_forward(h, Wd, bd, xd, compute="f32")
    loss, dy = rt.rtr_mlp_tr_loss(h, y, xd, SMALL_K, SMALL_R, 1.0 / B)
    dW, db = rt.rtr_mlp_backward(h, Wd, xd, acts, dy, compute="f32")
    params = [(w.astype(np.float64), c.astype(np.float64)) for w, c in zip(W, b)]
    grads = om.backward(params, x.astype(np.float64), x.astype(np.float64), SMALL_K, SMALL_R)
    assert abs(float(loss.mean()) - om.loss(params, x.astype(np.float64), x.astype(np.float64),
                                            SMALL_K, SMALL_R)) < 1e-5
    for l, (gW, gb) in enumerate(grads):
        assert rel(dW[l].cpu().numpy(), gW) < 1e-4, l
        assert rel(db[l].cpu().numpy(), gb) < 1e-4, l


def test_adam_matches_oracle(h):
    rng = np.random.default_rng(8)
    w = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    wd, md, vd = (torch.as_tensor(a).to(DEV) for a in (w, m, v))
    wo, mo, vo = w.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(1000).astype(np.float32)
        rt.rtr_mlp_adam(h, wd, torch.as_tensor(g).to(DEV), md, vd, t, lr=1e-2)
        wo, mo, vo = om.adam_step(wo, g.astype(np.float64), mo, vo, t, lr=1e-2)
    assert rel(wd.cpu().numpy(), wo) < 1e-6
    assert rel(vd.cpu().numpy(), vo) < 1e-5


def test_to_cores(h):
    y = torch.randn(3, 768, device=DEV)
    Z = rt.rtr_mlp_to_cores(h, y)
    assert torch.equal(Z.float(), y)
    pn2 = torch.tensor([16.0, 1.0, 81.0], dtype=torch.float64, device=DEV)
    Z = rt.rtr_mlp_to_cores(h, y, pn2, order=4).cpu().numpy()
    want = y.double().cpu().numpy() * np.array([2.0, 1.0, 3.0])[:, None] ** 0.5
    np.testing.assert_allclose(Z, want, rtol=1e-14)


@pytest.mark.parametrize("compute,tol", [("f32", 1e-4), ("bf16", 2e-2)])
@pytest.mark.parametrize("full", [False, True])
def test_backward_precisions_and_full_size(h, compute, tol, full):
    """Backward pass in both precisions, on a small network and on the full warm-start network
    (12^4 = 20736 inputs -> 1024 -> 1024 -> 1024 -> 768 outputs, the 4 cores 4 x 12 x 4).

    FP32: the whole chain (forward, TR loss, backward) against the oracle's gradients of the
    mean loss.  bf16: every product rounds both operands to 8 significant bits; the TR loss
    derivative is cubic in the network's output, so the output's bf16 error is amplified on the
    way into the backward pass.  The backward kernels are therefore compared stage-wise: the
    oracle's back-propagation (FP64) applied to the GPU's own layer inputs and output gradient,
    at the per-product bf16 accuracy 2e-2 of the forward test; the loss at 2e-2 as well."""
    K, R = (C5_K, C5_R) if full else (SMALL_K, SMALL_R)
    out = sum(a * b * c for a, b, c in om.core_shapes(K, R))
    sizes = [int(np.prod(K)), 1024, 1024, 1024, out] if full else [72, 64, 48, out]
    B = 8
    say("mlp backward", compute, "full" if full else "small")
    W, b = net(sizes, 16 if full else 6)
    P, x = inputs(B, K, 17)
    Wd, bd, xd = to_dev(W), to_dev(b), torch.as_tensor(x).to(DEV)
    y, acts = rt.rtr_mlp_forward(h, Wd, bd, xd, compute=compute)
    loss, dy = rt.rtr_mlp_tr_loss(h, y, xd, K, R, 1.0 / B)
    dW, db = rt.rtr_mlp_backward(h, Wd, xd, acts, dy, compute=compute)
    params = [(w.astype(np.float64), c.astype(np.float64)) for w, c in zip(W, b)]
    lo = om.loss(params, x.astype(np.float64), x.astype(np.float64), K, R)
    say("  loss", float(loss.mean()), lo)
    assert abs(float(loss.mean()) - lo) <= (1e-5 if compute == "f32" else tol) * max(1.0, abs(lo))
    if compute == "f32":
        grads = om.backward(params, x.astype(np.float64), x.astype(np.float64), K, R)
    else:
        a_in = [x.astype(np.float64)] + [t.cpu().numpy().astype(np.float64) for t in acts]
        grads = om.backprop(params, a_in, dy.cpu().numpy().astype(np.float64))
    for l, (gW, gb) in enumerate(grads):
        eW, eb = rel(dW[l].cpu().numpy(), gW), rel(db[l].cpu().numpy(), gb)
        say("  layer", l, f"dW {eW:.3g} db {eb:.3g}")
        assert eW < tol and eb < tol, (l, eW, eb)


def test_core_loss_matches_oracle(h):
    """Supervised core loss and its gradient against the oracle's definition."""
    rng = np.random.default_rng(21)
    y = rng.standard_normal((5, 768)).astype(np.float32)
    t = rng.standard_normal((5, 768)).astype(np.float32)
    loss, dy = rt.rtr_mlp_core_loss(h, torch.as_tensor(y).to(DEV), torch.as_tensor(t).to(DEV), 0.2)
    lo, go = om.core_loss(y.astype(np.float64), t.astype(np.float64), 0.2)
    assert rel(loss.cpu().numpy(), lo) < 1e-6
    assert rel(dy.cpu().numpy(), go) < 1e-6
