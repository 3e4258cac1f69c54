"""isax_query_noalloc: the query entry point that allocates no device memory (GPU).

Its answers must equal those of isax_query_ex on the same inputs (ids, and
distance bits, since both run the same kernels in the same order), and the
exact answers of the FP64 oracle; two calls in a row, the second smaller,
share the fixed per-device array.  The library's allocation fault injection
counts every allocation request of the library, so a no-allocation call must
succeed with it armed; device free memory must not move across a call.
Sizes beyond the array are rejected before any device work.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu

RTOL = 1e-4


def say(*a):
    print("[noalloc]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    X = workload.random_walks(50_021, 256, seed=20090171, device="cuda")
    Q, _, _ = workload.noisy_queries(X, 40, seed=20091172)
    Q = Q.cuda()
    idx = isax.Index(X, 16, 8, precision=3)
    ref_ids, ref_d2 = kr.knn_exact_c(X.cpu().numpy(), Q.cpu().numpy(), 10)
    yield {"isax": isax, "X": X, "Q": Q, "idx": idx, "ids": ref_ids, "d2": ref_d2}
    idx.close()


def _raw(isax, idx, Q, k, noalloc, **kw):
    """One call through the C ABI; returns (rc, ids, dists) with outputs pre-filled by a marker."""
    m = Q.shape[0]
    ids = torch.full((m, k), -7, dtype=torch.int64, device="cuda")
    d = torch.full((m, k), 7.0, dtype=torch.float32, device="cuda")
    opt = isax.QueryOptions(isax.MODES[kw.get("mode", "index")], kw.get("cap", 0), kw.get("flags", 0),
                            kw.get("batch", 0), None, isax._stream(None), None,
                            isax.METRICS[kw.get("metric", "ed")], kw.get("window", 0), kw.get("hybrid_leaves", 0))
    fn = isax.lib().isax_query_noalloc if noalloc else isax.lib().isax_query_ex
    rc = fn(idx.handle, Q.data_ptr(), m, k, ids.data_ptr(), d.data_ptr(), ctypes.byref(opt))
    torch.cuda.synchronize()
    return rc, ids, d


CASES = [dict(mode="index"), dict(mode="scan"), dict(mode="bf16"), dict(mode="fp8"), dict(mode="hybrid"),
         dict(mode="hybrid", hybrid_leaves=1), dict(mode="index", batch=16), dict(mode="bf16", batch=7),
         dict(mode="index", cap=12), dict(mode="index", metric="dtw", window=6), dict(mode="index", flags=7)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_two_calls_match_query_ex_and_the_oracle(setup, case):
    isax, idx = setup["isax"], setup["idx"]
    for Q, k in ((setup["Q"], 10), (setup["Q"][3:10].contiguous(), 3)):
        say(case, "m =", Q.shape[0], "k =", k)
        rc0, ids0, d0 = _raw(isax, idx, Q, k, False, **case)
        assert rc0 == isax.ISAX_OK, isax.last_error()
        rc1, ids1, d1 = _raw(isax, idx, Q, k, True, **case)
        assert rc1 == isax.ISAX_OK, isax.last_error()
        assert torch.equal(ids1, ids0)
        assert torch.equal(d1.view(torch.int32), d0.view(torch.int32))
        if case.get("metric", "ed") == "ed":
            rows = slice(0, 40) if Q.shape[0] == 40 else slice(3, 10)
            ref_ids, ref_d = setup["ids"][rows, :k], np.sqrt(setup["d2"][rows, :k])
            assert np.array_equal(ids1.cpu().numpy(), ref_ids)
            got = d1.cpu().numpy().astype(np.float64)
            assert np.all(np.abs(got - ref_d) <= RTOL * np.maximum(ref_d, 1e-30))


def test_no_allocation_request_and_no_device_memory_change(setup):
    isax, idx, Q = setup["isax"], setup["idx"], setup["Q"]
    rc, ids0, d0 = _raw(isax, idx, Q, 10, True, mode="hybrid", hybrid_leaves=1)  # warm
    assert rc == isax.ISAX_OK
    for mode in ["index", "bf16", "hybrid"]:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        isax.debug_fail_allocation(1)  # the next allocation request of the library fails
        try:
            rc, ids1, d1 = _raw(isax, idx, Q, 10, True, mode=mode, hybrid_leaves=1)
        finally:
            isax.debug_fail_allocation(0)
        assert rc == isax.ISAX_OK, (mode, isax.last_error())
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (mode, free0, free1)
        assert torch.equal(ids1, ids0)
        # the same call through isax_query_ex does allocate: the armed injection makes it fail
        isax.debug_fail_allocation(1)
        try:
            rc, _, _ = _raw(isax, idx, Q, 10, False, mode=mode, hybrid_leaves=1)
        finally:
            isax.debug_fail_allocation(0)
        assert rc == isax.ISAX_ENOMEM


def test_sizes_beyond_the_array_are_rejected_before_device_work(setup):
    isax, idx = setup["isax"], setup["idx"]
    # staged answers alone: 30000 x 1024 x 12 bytes > 256 MiB
    Qbig = setup["Q"][:1].repeat(30000, 1).contiguous()
    rc, ids, d = _raw(isax, idx, Qbig, 1024, True, mode="scan")
    assert rc == isax.ISAX_EINVAL and "isax_query_noalloc" in isax.last_error(), isax.last_error()
    assert bool((ids == -7).all()) and bool((d == 7.0).all())
    # an explicit batch whose filter scratch does not fit (about 1 MiB of candidates per query)
    Q1k = setup["Q"][:1].repeat(1024, 1).contiguous()
    rc, ids, d = _raw(isax, idx, Q1k, 10, True, mode="bf16", batch=1024)
    assert rc == isax.ISAX_EINVAL and "batches of 1024" in isax.last_error(), isax.last_error()
    assert bool((ids == -7).all())
    # the same queries with the batch chosen by the library fit, in several batches
    rc, ids, d = _raw(isax, idx, Q1k, 10, True, mode="bf16")
    assert rc == isax.ISAX_OK, isax.last_error()
    assert bool((ids == ids[0]).all())
    ref = setup["ids"][0, :10]
    assert np.array_equal(ids[0].cpu().numpy(), ref)
