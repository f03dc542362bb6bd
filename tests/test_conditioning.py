"""The conditioning probe composes the oracle's steps without changing them: with no
perturbation it reproduces the oracle's whole run exactly, and its amplification factors
are stable in the linear regime (half the perturbation, half the change)."""
import numpy as np

import conditioning as C
from oracle import rtr as orc
import workloads as W


def _case():
    w = W.Workload("cond", [9, 8, 10, 7], [2, 2, 2, 2], [5, 4, 5, 4], 1, 6, 30.0, 77)
    X, _ = W.make_tensor(w)
    return w, X.numpy(), W.make_init(w)


def test_probe_without_perturbation_is_the_oracle():
    w, X, Z0 = _case()
    ref = orc.rtr_als(X, w.K, Z0, w.sweeps, q=w.q, seed=w.seed)
    got = C.perturbed_rtr_als(X, w.K, Z0, w.sweeps, w.q, w.seed, 0.0, np.random.default_rng(0))
    for a, b in zip(got["Q"], ref["Q"]):
        assert np.array_equal(a, b)
    assert np.array_equal(got["P"], ref["P"])
    assert np.array_equal(got["rse_trace"], ref["rse_trace"])
    assert got["rse"] == ref["rse"]


def test_probe_is_linear_in_the_perturbation():
    w, X, Z0 = _case()
    base = C.quantities(orc.rtr_als(X, w.K, Z0, w.sweeps, q=w.q, seed=w.seed))
    ch = []
    for d in (1e-8, 5e-9):
        r = C.quantities(C.perturbed_rtr_als(X, w.K, Z0, w.sweeps, w.q, w.seed, d,
                                             np.random.default_rng(5)))
        ch.append(C.distance(r["P"], base["P"], "P"))
    assert 0.45 < ch[1] / ch[0] < 0.55
