"""Extensions beyond the in-HBM random-walk collections, same exactness bar.

* Embedding vectors (high-dimensional, not z-normalised): the index, the
  reduced-precision filter and the scan all return the oracle's answer.
* Raw data larger than device memory: the collection stays in pinned host
  memory (the library borrows the pointer and reads it over the bus); only the
  summaries, the leaf layout and the query state live in HBM.
"""
import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isax():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    return isax


@pytest.mark.parametrize("dim", [128, 384])
def test_embedding_vectors(isax, dim):
    g = torch.Generator(device="cuda").manual_seed(dim)
    # clustered embeddings: 200 centres, anisotropic spread, not normalised
    centres = torch.randn(200, dim, device="cuda", generator=g) * 3.0
    lab = torch.randint(0, 200, (60_000,), device="cuda", generator=g)
    X = (centres[lab] + torch.randn(60_000, dim, device="cuda", generator=g) * 0.7).float().contiguous()
    Q = (centres[torch.randint(0, 200, (24,), device="cuda", generator=g)] +
         torch.randn(24, dim, device="cuda", generator=g) * 0.7).float().contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(X.cpu().numpy(), Q.cpu().numpy(), 10)
    idx = isax.Index(X, 16, 8, precision=3)
    for mode in ("index", "scan", "bf16", "fp8"):
        ids, d = idx.query(Q, k=10, mode=mode)
        assert np.array_equal(ids.cpu().numpy(), ref_ids), mode
        assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0), mode


def test_raw_data_in_pinned_host_memory(isax):
    Xd = workload.random_walks(200_003, 256, seed=61, device="cuda")
    Xh = torch.empty(Xd.shape, dtype=torch.float32, pin_memory=True)
    Xh.copy_(Xd.cpu())
    del Xd
    Qn, _, _ = workload.noisy_queries(Xh.cuda(), 12, seed=62)
    Q = Qn.contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(Xh.numpy(), Q.cpu().numpy(), 5)
    import ctypes
    # the index borrows the host pointer; build and queries read it from the device
    opt = isax.BuildOptions(0, 0, 0, 0, None)
    h = isax.lib().isax_build_ex(Xh.data_ptr(), Xh.shape[0], 256, 16, 8, ctypes.byref(opt))
    assert h, isax.last_error()
    try:
        for mode in (isax.MODE_INDEX, isax.MODE_SCAN):
            ids = torch.empty((12, 5), dtype=torch.int64, device="cuda")
            d = torch.empty((12, 5), dtype=torch.float32, device="cuda")
            qo = isax.QueryOptions(mode, 0, 0, 0, None, None, None)
            rc = isax.lib().isax_query_ex(ctypes.c_void_p(h), Q.data_ptr(), 12, 5, ids.data_ptr(), d.data_ptr(),
                                          ctypes.byref(qo))
            assert rc == 0, isax.last_error()
            assert np.array_equal(ids.cpu().numpy(), ref_ids)
            assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0)
    finally:
        isax.lib().isax_free(ctypes.c_void_p(h))
