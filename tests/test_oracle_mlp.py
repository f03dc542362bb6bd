"""Pins of the FP64 warm-start MLP oracle (CPU only)."""
import numpy as np

from oracle import mlp
from oracle.tensor import tr_full

K, R = (3, 4, 2, 3), (2, 3, 2, 2)
DIN = int(np.prod(K))
DOUT = sum(a * b * c for a, b, c in mlp.core_shapes(K, R))


def make_params(sizes, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return [(scale * rng.standard_normal((a, b)), 0.1 * rng.standard_normal(b))
            for a, b in zip(sizes[:-1], sizes[1:])]


def brute_psi(cores):
    """Eq. (1) entry by entry: trace of the product of the slices."""
    dims = [c.shape[1] for c in cores]
    out = np.zeros(dims)
    for idx in np.ndindex(*dims):
        M = np.eye(cores[0].shape[0])
        for c, i in zip(cores, idx):
            M = M @ c[:, i, :]
        out[idx] = np.trace(M)
    return out


def test_psi_batch_matches_brute_force():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((2, DOUT))
    got = mlp.psi_batch(y, K, R)
    for s in range(2):
        want = brute_psi(mlp.unpack_cores(y[s], K, R)).reshape(-1)
        np.testing.assert_allclose(got[s], want, rtol=1e-12, atol=1e-12)


def test_core_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    cores = [rng.standard_normal(s) for s in mlp.core_shapes(K, R)]
    G = rng.standard_normal(K)
    grads = mlp._psi_grad_cores(cores, G)
    h = 1e-6
    for n in range(4):
        for _ in range(5):
            idx = tuple(rng.integers(0, d) for d in cores[n].shape)
            cp = [c.copy() for c in cores]
            cm = [c.copy() for c in cores]
            cp[n][idx] += h
            cm[n][idx] -= h
            fd = (np.sum(G * tr_full(cp)) - np.sum(G * tr_full(cm))) / (2 * h)
            assert abs(fd - grads[n][idx]) < 1e-7 * max(1.0, abs(fd))


def test_backward_by_central_differences():
    sizes = [DIN, 16, 12, DOUT]
    params = make_params(sizes, 3)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, DIN))
    P = rng.standard_normal((3, DIN))
    grads = mlp.backward(params, x, P, K, R)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for which, arr in (("W", W), ("b", b)):
            g = grads[l][0] if which == "W" else grads[l][1]
            for _ in range(6):
                idx = tuple(rng.integers(0, d) for d in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(params, x, P, K, R)
                arr[idx] = old - h
                lm = mlp.loss(params, x, P, K, R)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(fd)), (l, which, idx, fd, g[idx])


def test_zero_loss_at_an_exact_fit():
    """Output layer zero, bias = packed cores with ||Psi|| = 1, target P = any positive
    multiple of Psi: loss and every gradient vanish."""
    rng = np.random.default_rng(5)
    cores = [rng.standard_normal(s) for s in mlp.core_shapes(K, R)]
    cores[0] /= np.linalg.norm(tr_full(cores))
    y = np.concatenate([c.reshape(-1) for c in cores])
    sizes = [DIN, 8, DOUT]
    params = make_params(sizes, 6)
    params[-1] = (np.zeros((8, DOUT)), y.copy())
    x = rng.standard_normal((2, DIN))
    P = np.stack([3.0 * tr_full(cores).reshape(-1), 0.5 * tr_full(cores).reshape(-1)])
    assert mlp.loss(params, x, P, K, R) < 1e-28
    for dW, db in mlp.backward(params, x, P, K, R):
        assert np.max(np.abs(dW)) < 1e-13 and np.max(np.abs(db)) < 1e-13


def test_adam_step_written_out():
    w, g = np.array([1.0, -2.0]), np.array([0.5, 0.25])
    m, v = np.zeros(2), np.zeros(2)
    w1, m1, v1 = mlp.adam_step(w, g, m, v, 1, lr=0.1)
    # step 1: mhat = g, vhat = g^2, update = lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    w2, m2, v2 = mlp.adam_step(w1, g, m1, v1, 2, lr=0.1)
    # step 2 with the same gradient: m2 = 0.19 g, v2 = 0.001999 g^2, and the bias corrections
    # 1 - 0.9^2 = 0.19, 1 - 0.999^2 = 0.001999 give mhat = g, vhat = g^2 again
    np.testing.assert_allclose(m2, 0.19 * g, rtol=1e-14)
    np.testing.assert_allclose(v2, 0.001999 * g * g, rtol=1e-12)
    np.testing.assert_allclose(w2, w1 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
