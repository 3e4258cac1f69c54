"""GPU parity of DTW k-NN on the iSAX index (and the plain DTW scan) against
the FP64 DTW oracle, through the C ABI.  Bars: ids bit-exact, distances within
1e-4 relative of the oracle."""
import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu

RTOL = 1e-4


@pytest.fixture(scope="module")
def isax():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    return isax


def _cpu(t):
    return t.detach().cpu().numpy()


def _check(ids, dists, ref_ids, ref_d2, k):
    ids, dists = _cpu(ids), _cpu(dists)
    assert np.array_equal(ids, ref_ids[:, :k]), (ids, ref_ids[:, :k])
    ref = np.sqrt(ref_d2[:, :k])
    err = np.abs(dists.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    err[ref == 0] = np.abs(dists[ref == 0])
    assert err.max() <= RTOL, err.max()


@pytest.fixture(scope="module")
def coll(isax):
    # several leaf tiles at leaf size 64 and a ragged tail
    X = workload.random_walks(30_011, 128, seed=7001, device="cuda")
    workload.planted_duplicates(X, [(29_999, 11)])
    Qn, _, _ = workload.noisy_queries(X, 6, seed=7002)
    Qf = workload.fresh_queries(2, 128, seed=7003, device="cuda")
    Q = torch.cat([Qn, Qf, X[11:12].clone()]).contiguous()
    return {"X": X, "Q": Q, "Xh": _cpu(X), "Qh": _cpu(Q), "ref": {}}


def _ref(coll, r, k=10):
    if r not in coll["ref"]:
        coll["ref"][r] = kr.knn_dtw_c(coll["Xh"], coll["Qh"], k, r)
    return coll["ref"][r]


@pytest.mark.parametrize("r", [0, 3, 12, 20, 31])
@pytest.mark.parametrize("mode", ["index", "scan"])
def test_dtw_parity(isax, coll, r, mode):
    idx = isax.Index(coll["X"], 16, 8, leaf_size=64)
    ref_ids, ref_d2 = _ref(coll, r)
    for k in (1, 10):
        ids, d = idx.query(coll["Q"], k=k, mode=mode, metric="dtw", window=r)
        _check(ids, d, ref_ids, ref_d2, k)


def test_dtw_window_zero_is_euclidean(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    a = idx.query(coll["Q"], k=5, metric="dtw", window=0)
    b = idx.query(coll["Q"], k=5)
    assert torch.equal(a[0], b[0])
    assert torch.allclose(a[1], b[1], rtol=1e-5, atol=0)


def test_dtw_self_query_and_duplicates(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    ids, d = idx.query(coll["Q"][-1:].contiguous(), k=3, metric="dtw", window=8)
    assert list(_cpu(ids)[0][:2]) == [11, 29_999] and np.all(_cpu(d)[0][:2] == 0)


@pytest.mark.parametrize("flags", [1, 2, 4, 7])
def test_dtw_switches(isax, coll, flags):
    idx = isax.Index(coll["X"], 16, 8)
    ref_ids, ref_d2 = _ref(coll, 12)
    ids, d = idx.query(coll["Q"], k=10, metric="dtw", window=12, flags=flags)
    _check(ids, d, ref_ids, ref_d2, 10)


def test_dtw_overflow_fallback_and_per_query_k(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    ref_ids, ref_d2 = _ref(coll, 3)
    ids, d = idx.query(coll["Q"], k=10, metric="dtw", window=3, candidate_capacity=10)
    _check(ids, d, ref_ids, ref_d2, 10)
    kq = torch.tensor([1 + (i % 10) for i in range(coll["Q"].shape[0])], dtype=torch.int32)
    ids, d = idx.query(coll["Q"], k=10, metric="dtw", window=3, k_per_query=kq)
    ids = _cpu(ids)
    for i, kk in enumerate(kq.tolist()):
        assert np.array_equal(ids[i, :kk], ref_ids[i, :kk]) and np.all(ids[i, kk:] == -1)


def test_dtw_stats(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    r = 12
    _, _, st = idx.query(coll["Q"], k=1, metric="dtw", window=r, stats=True)
    n, L = coll["X"].shape
    for s in st:
        assert 0 < s["dtw_series"] <= n
        assert s["dtw_cells"] <= s["dtw_series"] * L * (2 * r + 1)
        assert s["leaves_kept"] <= s["leaves_scanned"]


@pytest.mark.parametrize("length,w,r", [(54, 6, 5), (54, 6, 20), (256, 16, 25), (96, 8, 31)])
def test_dtw_lengths(isax, length, w, r):
    X = workload.random_walks(6_007, length, seed=length, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 4, seed=length + 1)
    Q = torch.cat([Qn, workload.fresh_queries(2, length, seed=length + 2, device="cuda")]).contiguous()
    ref_ids, ref_d2 = kr.knn_dtw_c(_cpu(X), _cpu(Q), 5, r)
    idx = isax.Index(X, w, 8)
    for mode in ("index", "scan"):
        ids, d = idx.query(Q, k=5, mode=mode, metric="dtw", window=r)
        _check(ids, d, ref_ids, ref_d2, 5)


def test_dtw_small_collection_k_equals_n(isax):
    X = workload.random_walks(37, 64, seed=3, device="cuda")
    Q = workload.fresh_queries(3, 64, seed=4, device="cuda")
    ref_ids, ref_d2 = kr.knn_dtw_c(_cpu(X), _cpu(Q), 37, 6)
    idx = isax.Index(X, 16, 8, leaf_size=16)
    for mode in ("index", "scan"):
        ids, d = idx.query(Q, k=37, mode=mode, metric="dtw", window=6)
        _check(ids, d, ref_ids, ref_d2, 37)


def test_dtw_argument_errors(isax, coll):
    idx = isax.Index(coll["X"][:1000].contiguous(), 16, 8, precision=1)
    Q = coll["Q"][:2].contiguous()
    for kw, msg in ((dict(mode="bf16", metric="dtw", window=3), "DTW runs in"),
                    (dict(metric="dtw", window=32), "window must be"),
                    (dict(metric="ed", window=2), "window must be 0"),
                    (dict(metric=5), "unknown metric")):
        with pytest.raises(isax.IsaxError) as e:
            idx.query(Q, k=1, **kw)
        assert msg in str(e.value)
    X = workload.random_walks(64, 4096, seed=5, device="cuda")
    big = isax.Index(X, 16, 8, leaf_size=16)
    with pytest.raises(isax.IsaxError) as e:
        big.query(X[:1].contiguous(), k=1, metric="dtw", window=3)
    assert "at most 2048" in str(e.value)


@pytest.mark.parametrize("r", [12, 20])
def test_dtw_sorted_rows_copy(isax, coll, r):
    idx = isax.Index(coll["X"], 16, 8, leaf_size=64, precision=4)
    ref_ids, ref_d2 = _ref(coll, r)
    for mode in ("index", "scan"):
        ids, d = idx.query(coll["Q"], k=10, mode=mode, metric="dtw", window=r)
        _check(ids, d, ref_ids, ref_d2, 10)


@pytest.mark.parametrize("w,c", [(8, 4), (32, 2)])
def test_dtw_metamorphic_summaries(isax, coll, w, c):
    """Other segment counts and cardinalities give the same DTW answer."""
    idx = isax.Index(coll["X"], w, c)
    ref_ids, ref_d2 = _ref(coll, 12)
    ids, d = idx.query(coll["Q"], k=5, metric="dtw", window=12)
    _check(ids, d, ref_ids, ref_d2, 5)


@pytest.fixture(scope="module")
def wide(isax):
    X = workload.random_walks(12_007, 128, seed=7011, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 4, seed=7012)
    Q = torch.cat([Qn, workload.fresh_queries(2, 128, seed=7013, device="cuda")]).contiguous()
    return {"X": X, "Q": Q, "idx": isax.Index(X, 16, 8, leaf_size=64)}


@pytest.mark.parametrize("r", list(range(16, 32)))
def test_dtw_every_drain_width(isax, wide, r):
    # windows 16-31 drain their queued series with a band width fixed at compile time
    # (four widths per register class): each width against the oracle, both modes
    ref_ids, ref_d2 = kr.knn_dtw_c(_cpu(wide["X"]), _cpu(wide["Q"]), 5, r)
    for mode in ("index", "scan"):
        ids, d = wide["idx"].query(wide["Q"], k=5, mode=mode, metric="dtw", window=r)
        _check(ids, d, ref_ids, ref_d2, 5)
