"""The no-allocation sketch entry point (for callers that cannot allocate device memory)
against rtr_sketch, through the C ABI: the same kernels and order of operations, so the
outputs agree bit for bit; two calls in a row, the second smaller (the shared scratch keeps
the first call's contents), on the matrix-core passes (FP32, BF16 with a power iteration) and
the FP64 path; a request above the fixed scratch is refused before anything runs."""
import numpy as np
import pytest
import torch

import paper_1901_01652_amd as rt

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def h():
    hd = rt.Handle(0)
    yield hd
    hd.close()


@pytest.mark.parametrize("dtype,compute,q", [(torch.float32, "f32", 0), (torch.float32, "bf16", 1),
                                             (torch.float64, None, 1)])
def test_noalloc_matches_sketch(h, dtype, compute, q):
    print("noalloc", dtype, compute, q, flush=True)
    g = torch.Generator().manual_seed(3)
    for dims, K in (((48, 40, 36, 30), (9, 8, 7, 6)), ((20, 17, 13), (5, 4, 3))):
        X = torch.randn(dims, generator=g, dtype=torch.float64).to(dtype).to(DEV)
        ref = rt.rtr_sketch(h, X, K, q, seed=11, tensor_id=2, compute=compute)
        Q = torch.full((rt.q_size(dims, K),), float("nan"), dtype=torch.float64, device=DEV)
        rt.rtr_sketch_noalloc(h, X, K, Q, q, seed=11, tensor_id=2, compute=compute)
        torch.cuda.synchronize()
        assert torch.equal(Q, ref), (dims, float((Q - ref).abs().max()))
        for qn in rt.unpack(Q.cpu(), rt.q_shapes(dims, K)):
            qn = qn.numpy()
            assert np.max(np.abs(qn.T @ qn - np.eye(qn.shape[1]))) < 1e-12


def test_noalloc_refuses_requests_above_its_scratch(h):
    print("noalloc limit", flush=True)
    dims, K = (128, 128, 128), (64, 64, 64)
    X = torch.zeros(dims, dtype=torch.float64, device=DEV)
    Q = torch.zeros(rt.q_size(dims, K), dtype=torch.float64, device=DEV)
    with pytest.raises(rt.RtrError) as e:
        rt.rtr_sketch_noalloc(h, X, K, Q)
    assert e.value.code == 2 and "scratch" in str(e.value)
