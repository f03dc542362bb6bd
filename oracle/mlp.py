"""FP64 oracle of the learned warm start for TR-ALS: a multilayer perceptron maps the
normalised projected tensor P~ = P / ||P|| (flattened, row-major K_1 x .. x K_N) to the N
initial cores (packed (R_n, K_n, R_{n+1}), the layout the ALS takes), trained on
L = mean over the batch of ||P~ - Psi(Z)||^2 / ||P~||^2, Psi as in Eq. (1).

Test infrastructure only: imported by tests, the smoke check and the benchmark's CPU
baseline, never by the GPU package.

Network (a reading: the paper names no architecture; the layer sizes come with the
workload): hidden layers h_l = relu(h_{l-1} W_l + b_l), output y = h_{L-1} W_L + b_L, with
W_l stored (in x out) row-major.  Adam (Kingma & Ba 2015) updates the parameters.

Pins (tests): central finite differences of ``loss`` against ``backward``; the loss is zero
when P~ is exactly Psi of the predicted cores; ``psi`` equals the pinned Eq. (1)
evaluator; one Adam step against the update rule written out for a scalar.
"""
import numpy as np

from .tensor import tr_full


def core_shapes(K, R):
    N = len(K)
    return [(R[n], K[n], R[(n + 1) % N]) for n in range(N)]


def unpack_cores(y, K, R):
    """Split one packed output vector into the N cores."""
    out, off = [], 0
    for s in core_shapes(K, R):
        n = s[0] * s[1] * s[2]
        out.append(np.asarray(y[off:off + n], dtype=np.float64).reshape(s))
        off += n
    return out


def forward(params, x):
    """params: list of (W, b); x: (B, d_in).  Returns (y, activations) where activations[l]
    is the input of layer l (activations[0] = x)."""
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = h @ W + b
        h = np.maximum(z, 0.0) if l < L - 1 else z
        if l < L - 1:
            acts.append(h)
    return h, acts


def psi_batch(y, K, R):
    """Psi of the cores in every row of y: (B, prod K)."""
    return np.stack([tr_full(unpack_cores(row, K, R)).reshape(-1) for row in y])


def loss(params, x, P, K, R):
    """Mean over the batch of ||P~ - Psi(Z(x))||^2 / ||P~||^2 with P~ = P / ||P|| per row."""
    Pn = P / np.linalg.norm(P, axis=1, keepdims=True)
    y, _ = forward(params, x)
    D = psi_batch(y, K, R) - Pn
    return float(np.mean(np.sum(D * D, axis=1)))


def _psi_grad_cores(cores, G):
    """d/dZ_n of <G, Psi(Z)> for a single sample: for core n, contract G with the product of
    the other cores around the ring: dZ_n[a, i, b] = sum over the other indices of
    G[i_1 .. i_N] * (Z_{n+1}(i_{n+1}) .. Z_{n-1}(i_{n-1}))[b, a]."""
    N = len(cores)
    grads = []
    for n in range(N):
        order = [(n + t) % N for t in range(1, N)]
        # subchain S[(i_{n+1} .. i_{n-1}), b, a]
        S = cores[order[0]]                     # R_{n+1} x K x R
        S = np.transpose(S, (1, 0, 2))          # K x R_{n+1} x R
        for m in order[1:]:
            Zm = cores[m]                       # R x K_m x R'
            S = np.einsum("jbc,cid->jibd", S, Zm).reshape(-1, S.shape[1], Zm.shape[2])
        # G permuted to (n, n+1, .., n-1) and flattened over the others
        Gp = np.transpose(G, [n] + order).reshape(G.shape[n], -1)   # K_n x J
        grads.append(np.einsum("ij,jba->aib", Gp, S))
    return grads


def backward(params, x, P, K, R):
    """Gradients of ``loss`` w.r.t. every (W, b): list of (dW, db)."""
    B = x.shape[0]
    Pn = P / np.linalg.norm(P, axis=1, keepdims=True)
    y, acts = forward(params, x)
    dy = np.zeros_like(y)
    shape = tuple(K)
    for s in range(B):
        cores = unpack_cores(y[s], K, R)
        D = tr_full(cores) - Pn[s].reshape(shape)
        gc = _psi_grad_cores(cores, 2.0 * D / B)
        dy[s] = np.concatenate([g.reshape(-1) for g in gc])
    return backprop(params, acts, dy)


def backprop(params, acts, dy):
    """The layer-by-layer gradients given the layer inputs ``acts`` (acts[0] = x, acts[l] the
    ReLU output feeding layer l) and the gradient ``dy`` of the loss w.r.t. the output:
    dW_l = acts[l]^T g_l, db_l = sum over the batch of g_l, g_{l-1} = (g_l W_l^T) * [acts[l] > 0]."""
    grads = [None] * len(params)
    g = dy
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        h_in = acts[l]
        grads[l] = (h_in.T @ g, g.sum(axis=0))
        if l > 0:
            g = (g @ W.T) * (acts[l] > 0.0)
    return grads


def core_loss(y, T, grad_scale=1.0):
    """Supervised loss on the packed cores: per sample ||y - T||^2, and its gradient
    grad_scale * 2 (y - T)."""
    D = y - T
    return np.sum(D * D, axis=1), grad_scale * 2.0 * D


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t = 1, 2, ..); returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
