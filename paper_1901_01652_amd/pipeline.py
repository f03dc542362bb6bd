"""Algorithm 1 end to end through the C ABI (no arithmetic here: only the calls in order)."""
import torch

from . import (rtr_sketch, rtr_compress, rtr_decompose, rtr_backproject, rtr_residual, keff,
               pack)


def rtr_als(h, X, K, R, Z_init, sweeps, power_iters=0, seed=0, tensor_id=0, compute=None,
            tol=0.0, stream=None):
    """Sketch -> QR -> compress -> TR-ALS -> back-project.  ``Z_init`` is a packed device
    buffer or a list of host cores.  Returns a dict of device tensors."""
    dims = list(X.shape)
    if not torch.is_tensor(Z_init):
        Z_init = pack(Z_init, X.device)
    Q = rtr_sketch(h, X, K, power_iters, seed, tensor_id, compute, stream=stream)
    pn2 = torch.zeros(1, dtype=torch.float64, device=X.device)
    P = rtr_compress(h, X, K, Q, compute, p_norm2=pn2, stream=stream)
    Z, trace, nsw = rtr_decompose(h, P, R, Z_init, sweeps, tol, stream=stream)
    G = rtr_backproject(h, dims, K, R, Z, Q, stream=stream)
    return {"Q": Q, "P": P, "p_norm2": pn2, "Z": Z, "err_trace": trace, "sweeps_run": nsw, "G": G}


def rse(h, X, R, G, stream=None):
    """Sec. 4 RSE = ||X - Psi(G)|| / ||X|| from the explicit residual kernel."""
    out = rtr_residual(h, X, R, G, stream=stream)
    o = out.cpu()
    return float((o[0] / o[1]).sqrt())
