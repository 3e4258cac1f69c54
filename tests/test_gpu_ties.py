"""Final ordering on near ties, wide tie windows, list growth and error paths (GPU).

Near ties (tests/near_ties.py): pairs and chains of series whose FP32
distances are equal or inverted against their exact order; the FP64 oracle
decides, and every mode must return its ids (the compensated recompute of the
window, Sec. II Similarity Search with ties by lower id).  The host test of
the same construction shows that a plain FP32 order gets these cases wrong.

Wide windows: thousands of exact duplicates of a query tie at the k-th
distance; the lowest ids must come back, also when the candidate list has to
grow.  Error paths: every device allocation of a query (and of a build) is
made to fail in turn; the call reports ENOMEM, the outputs stay untouched,
and nothing leaks.
"""
import sys

import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr
from tests import near_ties as nt

pytestmark = pytest.mark.gpu

RTOL = 1e-4


def say(*a):
    print("[ties]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def isax():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    return isax


@pytest.fixture(scope="module")
def tied(isax):
    n = 100_003
    X = workload.random_walks(n, 256, seed=20090168, device="cuda")
    Xh = X.cpu().numpy()
    Qt, cases = nt.plant_cases(Xh, seed=20091168)
    Qn, _, _ = workload.noisy_queries(torch.from_numpy(Xh), 6, seed=20091169)
    Qh = np.concatenate([Qt, Qn.numpy()]).astype(np.float32)
    X.copy_(torch.from_numpy(Xh))
    # 12 columns: one case has nine planted series closer than its tied pair
    ids, d2 = kr.knn_exact_c(Xh, Qh, 12)
    for c in cases:  # the construction holds on this collection too
        m = len(c["closer"])
        assert ids[c["query"], m:m + len(c["ids"])].tolist() == c["ids"][::-1]
    idx = isax.Index(X, 16, 8, precision=3)
    yield {"X": X, "Q": torch.from_numpy(Qh).cuda(), "ids": ids, "d2": d2, "idx": idx, "cases": cases}
    idx.close()


def _check(ids, d, ref_ids, ref_d2, k):
    ids, d = ids.cpu().numpy(), d.cpu().numpy().astype(np.float64)
    assert np.array_equal(ids, ref_ids[:, :k]), (ids, ref_ids[:, :k])
    ref = np.sqrt(ref_d2[:, :k])
    assert np.all(np.abs(d - ref) <= RTOL * np.maximum(ref, 1e-30))


@pytest.mark.parametrize("k", [1, 2, 10])
@pytest.mark.parametrize("mode,extra", [("index", {}), ("scan", {}), ("bf16", {}), ("fp8", {}),
                                        ("hybrid", {}), ("hybrid", {"hybrid_leaves": 1}),
                                        ("hybrid", {"hybrid_leaves": 10 ** 9}),
                                        ("hybrid", {"flags": 8}), ("index", {"flags": 7})])
def test_near_ties_follow_the_exact_order(tied, mode, extra, k):
    say(mode, extra, "k =", k)
    ids, d = tied["idx"].query(tied["Q"], k=k, mode=mode, **extra)
    _check(ids, d, tied["ids"], tied["d2"], k)


def test_near_ties_with_grown_candidate_lists(tied):
    # a list of k slots overflows at once: the re-run grows it and still orders the window
    ids, d, st = tied["idx"].query(tied["Q"], k=10, mode="index", candidate_capacity=10, stats=True)
    _check(ids, d, tied["ids"], tied["d2"], 10)
    assert max(s["candidate_capacity"] for s in st) > 10


# ----------------------------------------------------------------------------- wide windows
@pytest.fixture(scope="module")
def dups(isax):
    n = 60_001
    X = workload.random_walks(n, 256, seed=20090169, device="cuda")
    rng = np.random.default_rng(20091170)
    dup = np.sort(rng.choice(n, size=3000, replace=False))
    src = int(dup[0])
    X[torch.as_tensor(dup[1:], device="cuda")] = X[src].clone()
    q_same = X[src:src + 1].clone()
    q_noisy, _, _ = workload.noisy_queries(X[src:src + 1].contiguous(), 1, seed=20091171, sigmas=(0.5,))
    Q = torch.cat([q_same, q_noisy.to(X.device)]).contiguous()
    idx = isax.Index(X, 16, 8, precision=3)
    yield {"X": X, "Q": Q, "dup": dup, "idx": idx}
    idx.close()


@pytest.mark.parametrize("mode", ["index", "scan", "bf16", "fp8", "hybrid"])
@pytest.mark.parametrize("k,cap", [(1, 0), (10, 0), (1024, 0), (10, 1000)])
def test_thousands_of_exact_ties_return_the_lowest_ids(dups, mode, k, cap):
    say("duplicates", mode, "k =", k, "cap =", cap)
    ids, d = dups["idx"].query(dups["Q"], k=k, mode=mode, candidate_capacity=cap)
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    want = dups["dup"][:k]
    assert np.array_equal(ids[0], want) and np.all(d[0] == 0)
    assert np.array_equal(ids[1], want) and np.all(d[1] == d[1, 0]) and d[1, 0] > 0
    ref = np.sqrt(kr.sq_dists(dups["X"][int(want[0]):int(want[0]) + 1].cpu().numpy(), dups["Q"][1].cpu().numpy()))
    assert abs(d[1, 0] - ref[0]) <= RTOL * ref[0]


# ----------------------------------------------------------------------------- error paths
def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_every_failed_allocation_leaves_outputs_untouched(isax, tied):
    idx, Q = tied["idx"], tied["Q"]
    m = Q.shape[0]
    for mode in ["index", "hybrid", "bf16"]:
        ref_ids, ref_d = idx.query(Q, k=10, mode=mode, batch=4, flags=8)
        _check(ref_ids, ref_d, tied["ids"], tied["d2"], 10)
        base = _free_bytes()
        failed = 0
        for n in range(1, 400):
            out_ids = torch.full((m, 10), -7, dtype=torch.int64, device="cuda")
            out_d = torch.full((m, 10), 7.0, dtype=torch.float32, device="cuda")
            isax.debug_fail_allocation(n)
            opt = isax.QueryOptions(isax.MODES[mode], 0, 8, 4, None, isax._stream(None), None, 0, 0, 0)
            rc = isax.lib().isax_query_ex(idx.handle, Q.data_ptr(), m, 10, out_ids.data_ptr(), out_d.data_ptr(),
                                          opt)
            isax.debug_fail_allocation(0)
            if rc == isax.ISAX_OK:
                assert torch.equal(out_ids, ref_ids) and torch.equal(out_d.view(torch.int32), ref_d.view(torch.int32))
                break
            failed += 1
            assert rc == isax.ISAX_ENOMEM and "injected" in isax.last_error(), (mode, n, rc, isax.last_error())
            assert bool((out_ids == -7).all()) and bool((out_d == 7.0).all()), (mode, n)
        else:
            pytest.fail("the query kept failing")
        say(mode, "allocation sites failed in turn:", failed)
        assert failed >= 10  # several batches, each with several allocations
        # no leak: the library works and holds no more memory than before
        ids, d = idx.query(Q, k=10, mode=mode, batch=4, flags=8)
        assert torch.equal(ids, ref_ids)
        assert _free_bytes() >= base - (64 << 20)


def test_failed_builds_free_what_they_allocated(isax, tied):
    X = tied["X"][:20_000].contiguous()
    base = _free_bytes()
    for n in range(1, 200):
        isax.debug_fail_allocation(n)
        try:
            idx = isax.Index(X, 16, 8, precision=3)
        except isax.IsaxError as e:
            assert "injected" in str(e)
            continue
        finally:
            isax.debug_fail_allocation(0)
        idx.close()
        break
    else:
        pytest.fail("the build kept failing")
    assert n > 5
    assert _free_bytes() >= base - (64 << 20)
