"""Algorithm 1 end to end through the C ABI (no arithmetic here: only the calls in order)."""
import torch

from . import (rtr_sketch, rtr_compress, rtr_decompose, rtr_backproject, rtr_residual, keff,
               pack)


def rtr_als(h, X, K, R, Z_init, sweeps, power_iters=0, seed=0, tensor_id=0, compute=None,
            tol=0.0, stream=None, projection="gaussian"):
    """Sketch -> QR -> compress -> TR-ALS -> back-project.  ``Z_init`` is a packed device
    buffer or a list of host cores.  ``projection``: "gaussian" (Alg. 1 as printed),
    "khatri_rao" (structured test matrices) or "sequential" (step 7 read sequentially).
    Returns a dict of device tensors."""
    dims = list(X.shape)
    if not torch.is_tensor(Z_init):
        Z_init = pack(Z_init, X.device)
    pn2 = torch.zeros(1, dtype=torch.float64, device=X.device)
    if projection == "sequential":
        from . import rtr_sketch_sequential
        if power_iters:
            raise ValueError("the sequential reading takes no power iterations")
        Q, P = rtr_sketch_sequential(h, X, K, seed, tensor_id, compute, p_norm2=pn2, stream=stream)
    else:
        Q = rtr_sketch(h, X, K, power_iters, seed, tensor_id, compute, stream=stream,
                       projection=projection)
        P = rtr_compress(h, X, K, Q, compute, p_norm2=pn2, stream=stream)
    Z, trace, nsw = rtr_decompose(h, P, R, Z_init, sweeps, tol, stream=stream)
    G = rtr_backproject(h, dims, K, R, Z, Q, stream=stream)
    return {"Q": Q, "P": P, "p_norm2": pn2, "Z": Z, "err_trace": trace, "sweeps_run": nsw, "G": G}


def rtr_als_coo(h, indices, values, dims, K, R, Z_init, sweeps, seed=0, tensor_id=0, tol=0.0,
                stream=None):
    """rTR-ALS of a tensor given by its nonzeros (``indices`` nnz x N int64, ``values``, on
    the device): sketch -> QR -> compress -> TR-ALS -> back-project, all in FP64.  Returns a
    dict of device tensors with ||X||^2 (``x_norm2``) and ||P||^2 (``p_norm2``), from which
    the RSE follows by the Pythagorean identity."""
    from . import rtr_sketch_coo, rtr_compress_coo
    dev = values.device
    if not torch.is_tensor(Z_init):
        Z_init = pack(Z_init, dev)
    xn2 = torch.zeros(1, dtype=torch.float64, device=dev)
    pn2 = torch.zeros(1, dtype=torch.float64, device=dev)
    Q = rtr_sketch_coo(h, indices, values, dims, K, seed, tensor_id, x_norm2=xn2, stream=stream)
    P = rtr_compress_coo(h, indices, values, dims, K, Q, p_norm2=pn2, stream=stream)
    Z, trace, nsw = rtr_decompose(h, P, R, Z_init, sweeps, tol, stream=stream)
    G = rtr_backproject(h, list(dims), K, R, Z, Q, stream=stream)
    return {"Q": Q, "P": P, "x_norm2": xn2, "p_norm2": pn2, "Z": Z, "err_trace": trace,
            "sweeps_run": nsw, "G": G}


def rse(h, X, R, G, stream=None):
    """Sec. 4 RSE = ||X - Psi(G)|| / ||X|| from the explicit residual kernel."""
    out = rtr_residual(h, X, R, G, stream=stream)
    o = out.cpu()
    return float((o[0] / o[1]).sqrt())


def rtr_svd(h, X, K, Rcap, eps, power_iters=0, seed=0, tensor_id=0, compute=None, stream=None):
    """rTR-SVD: sketch -> QR -> compress -> TR-SVD (ranks chosen for ||P - Psi(Z)|| <= eps ||P||)
    -> back-project.  ``Rcap`` caps the ranks (it sizes the outputs).  Returns a dict of device
    tensors plus the chosen ranks (host list)."""
    from . import rtr_decompose_svd, svd_cores
    dims = list(X.shape)
    Q = rtr_sketch(h, X, K, power_iters, seed, tensor_id, compute, stream=stream)
    pn2 = torch.zeros(1, dtype=torch.float64, device=X.device)
    P = rtr_compress(h, X, K, Q, compute, p_norm2=pn2, stream=stream)
    Z, ranks, err = rtr_decompose_svd(h, P, Rcap, eps, stream=stream)
    R = [int(r) for r in ranks.cpu()]
    Kp = keff(dims, K)
    Zc = pack(svd_cores(Z, R, Kp, Rcap), X.device)
    G = rtr_backproject(h, dims, K, R, Zc, Q, stream=stream)
    return {"Q": Q, "P": P, "p_norm2": pn2, "Z": Zc, "ranks": R, "p_err": err, "G": G}


def tr_als_full(h, X, R, Z_init, sweeps, tol=0.0, stream=None):
    """The traditional counterpart of rTR-ALS: TR-ALS on the full tensor (no projection; the
    per-sweep error is then the RSE itself).  X is handed to the decomposition in FP64 (a
    format conversion; the decomposition's arithmetic is the library's)."""
    if not torch.is_tensor(Z_init):
        Z_init = pack(Z_init, X.device)
    P = X if X.dtype == torch.float64 else X.to(torch.float64)
    Z, trace, nsw = rtr_decompose(h, P, R, Z_init, sweeps, tol, stream=stream)
    return {"Z": Z, "err_trace": trace, "sweeps_run": nsw}


def tr_svd_full(h, X, Rcap, eps, stream=None):
    """The traditional counterpart of rTR-SVD: TR-SVD on the full tensor (FP64)."""
    from . import rtr_decompose_svd
    P = X if X.dtype == torch.float64 else X.to(torch.float64)
    Z, ranks, err = rtr_decompose_svd(h, P, Rcap, eps, stream=stream)
    return {"Z": Z, "ranks": [int(r) for r in ranks.cpu()], "p_err": err}
