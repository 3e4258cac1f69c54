"""Hybrid mode: per query, the iSAX path or the BF16 filter, chosen by how many
leaves lie within the approximate answer's best-so-far.  Whatever the split,
the answer must equal the oracle's (ids bit-exact, distances within 1e-4
relative of FP64) and equal the other modes' answers bit for bit.
"""
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


@pytest.fixture(scope="module")
def coll(isax):
    # 391 leaves of 256 (two leaf tiles) and a ragged tail; queries of every noise level
    X = workload.random_walks(100_003, 256, seed=20090165, device="cuda")
    workload.planted_duplicates(X, [(99_998, 21), (40_000, 21)])
    Qn, _, sig = workload.noisy_queries(X, 150, seed=20091165)
    Q = torch.cat([Qn, workload.fresh_queries(6, 256, seed=20091166, device="cuda"), X[21:22].clone()]).contiguous()
    idx = isax.Index(X, 16, 8, precision=1)
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Q), 10)
    return {"X": X, "Q": Q, "idx": idx, "ids": ref_ids, "d2": ref_d2}


def _check(ids, d, ref_ids, ref_d2, k):
    ids, d = _cpu(ids), _cpu(d)
    assert np.array_equal(ids, ref_ids[:, :k])
    ref = np.sqrt(ref_d2[:, :k])
    err = np.abs(d.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    err[ref == 0] = np.abs(d[ref == 0])
    assert err.max() <= RTOL, err.max()


@pytest.mark.parametrize("k", [1, 10])
@pytest.mark.parametrize("limit", [0, 1, "p80", 10**9])
def test_hybrid_parity_any_split(isax, coll, k, limit):
    idx, Q = coll["idx"], coll["Q"]
    m = Q.shape[0]
    if limit == "p80":
        _, _, si = idx.query(Q, k=k, mode="index", stats=True)
        li = sorted(s["leaves_initial"] for s in si)
        limit = max(1, li[int(0.8 * m)])
    ids, d, st = idx.query(Q, k=k, mode="hybrid", hybrid_leaves=limit, stats=True)
    _check(ids, d, coll["ids"], coll["d2"], k)
    n_leaves = idx.info()["n_leaves"]
    li = np.array([s["leaves_initial"] for s in st])
    path = np.array([s["path"] for s in st])
    assert set(path.tolist()) <= {isax.MODE_INDEX, isax.MODE_BF16}
    if not limit:
        # a batch over 100K series: the filter alone is cheaper than the hybrid's own work
        assert np.all(path == isax.MODE_BF16) and np.all(li == -1)
    else:
        assert np.all((li >= 0) & (li < n_leaves))
        # round 1 only lowers the count a query is routed by: few leaves -> iSAX path
        assert np.all(path[li <= limit] == isax.MODE_INDEX)
    if limit == 10**9:
        assert np.all(path == isax.MODE_INDEX)


def test_hybrid_routes_near_to_index_and_far_to_filter(isax, coll):
    X = coll["X"]
    Qn, _, _ = workload.noisy_queries(X, 12, seed=20091168, sigmas=(0.01,))
    Qf = workload.fresh_queries(12, 256, seed=20091169, device="cuda")
    Q = torch.cat([Qn, Qf]).contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Q), 1)
    ids, d, st = coll["idx"].query(Q, k=1, mode="hybrid", hybrid_leaves=12, stats=True)
    _check(ids, d, ref_ids, ref_d2, 1)
    path = np.array([s["path"] for s in st])
    assert np.all(path[:12] == isax.MODE_INDEX)   # near copies: the index path
    assert np.any(path[12:] == isax.MODE_BF16)    # fresh walks: the filter
    # without a limit: the filter answers a batch over 100K series in less time
    # than the hybrid's own work, so the whole batch takes the BF16 path at once
    ids, d, st = coll["idx"].query(Q, k=1, mode="hybrid", stats=True)
    _check(ids, d, ref_ids, ref_d2, 1)
    assert all(s["path"] == isax.MODE_BF16 and s["leaves_initial"] == -1 for s in st)


def test_hybrid_equals_other_modes_bitwise(isax, coll):
    idx, Q = coll["idx"], coll["Q"]
    ih, dh = idx.query(Q, k=10, mode="hybrid")
    for mode in ("index", "bf16", "scan"):
        im, dm = idx.query(Q, k=10, mode=mode)
        assert torch.equal(ih, im), mode
        assert torch.equal(dh.view(torch.int32), dm.view(torch.int32)), mode


def test_hybrid_routes_by_noise(isax, coll):
    # near queries (sigma 0.01) keep few leaves under their first bound; sigma 1 keeps most
    X = coll["X"]
    Qn, _, sig = workload.noisy_queries(X, 30, seed=20091167)
    _, _, st = coll["idx"].query(Qn, k=1, mode="hybrid", hybrid_leaves=40, stats=True)
    sig = np.asarray(sig)
    li = np.array([s["leaves_initial"] for s in st])
    assert np.median(li[sig == 1.0]) > 4 * np.median(li[sig == 0.01]) + 4, (li, sig)


def test_hybrid_index_mode_reports_leaves_initial(isax, coll):
    idx, Q = coll["idx"], coll["Q"]
    _, _, sh = idx.query(Q, k=3, mode="hybrid", hybrid_leaves=40, stats=True)
    _, _, si = idx.query(Q, k=3, mode="index", stats=True)
    assert [s["leaves_initial"] for s in sh] == [s["leaves_initial"] for s in si]
    _, _, sb = idx.query(Q, k=3, mode="bf16", stats=True)
    assert all(s["leaves_initial"] == -1 and s["path"] == isax.MODE_BF16 for s in sb)
    _, _, sn = idx.query(Q, k=3, mode="index", flags=isax.QF_NO_BEST_FIRST, stats=True)
    assert all(s["leaves_initial"] == -1 and s["path"] == isax.MODE_INDEX for s in sn)


def test_hybrid_batches_per_query_k_and_overflow(isax, coll):
    idx, Q = coll["idx"], coll["Q"]
    m = Q.shape[0]
    kq = torch.tensor([1 + (7 * i) % 10 for i in range(m)], dtype=torch.int32, device="cuda")
    for opts in (dict(batch=17), dict(candidate_capacity=10), dict(batch=7, candidate_capacity=12),
                 dict(flags=isax.QF_NO_BEST_FIRST), dict(flags=3)):
        ids, d = idx.query(Q, k=10, mode="hybrid", k_per_query=kq, hybrid_leaves=1, **opts)
        ids, d = _cpu(ids), _cpu(d)
        for i in range(m):
            kk = int(kq[i])
            assert np.array_equal(ids[i, :kk], coll["ids"][i, :kk]), (opts, i)
            assert np.all(ids[i, kk:] == -1) and np.all(np.isinf(d[i, kk:]))
            ref = np.sqrt(coll["d2"][i, :kk])
            err = np.abs(d[i, :kk] - ref) / np.maximum(ref, 1e-30)
            err[ref == 0] = np.abs(d[i, :kk][ref == 0])
            assert err.max() <= RTOL


def test_hybrid_small_collection_and_errors(isax):
    X = workload.random_walks(700, 64, seed=61, device="cuda")
    Q = workload.noisy_queries(X, 9, seed=62)[0]
    ref_ids, _ = kr.knn_exact_c(_cpu(X), _cpu(Q), 700)
    idx = isax.Index(X, 16, 8, leaf_size=16, precision=1)
    for k in (1, 5, 700):
        for limit in (0, 1, 2, 10**6):
            ids, _ = idx.query(Q, k=k, mode="hybrid", hybrid_leaves=limit)
            assert np.array_equal(_cpu(ids), ref_ids[:, :k])
    plain = isax.Index(X, 16, 8)
    with pytest.raises(isax.IsaxError, match="BF16 copy"):
        plain.query(Q, k=1, mode="hybrid")
    with pytest.raises(isax.IsaxError, match="hybrid_leaves"):
        idx.query(Q, k=1, mode="hybrid", hybrid_leaves=-1)
    with pytest.raises(isax.IsaxError, match="DTW runs in"):
        idx.query(Q, k=1, mode="hybrid", metric="dtw", window=3)
    ids, _ = idx.query(Q[:0], k=1, mode="hybrid")
    assert ids.shape == (0, 1)


@pytest.mark.parametrize("k", [1, 10])
def test_leaves_initial_matches_oracle_envelope_bounds(isax, coll, k):
    # the leaf pass (with its node-level pruning) counts the leaves whose FP64 envelope
    # MINDIST is within the first best-so-far, up to the home leaf and rounding at the edge
    from oracle import isax_ref as ir
    idx, Q = coll["idx"], coll["Q"]
    _, _, st = idx.query(Q, k=k, mode="index", stats=True)
    _, _, lo, hi = (_cpu(t) for t in idx.export())
    paa = ir.paa64(_cpu(Q), 16)
    beta = ir.breakpoints(8)
    for j, s in enumerate(st):
        lb = ir.envelope_mindist_sq(paa[j], lo, hi, beta, 256 // 16)
        tau = float(s["tau_initial"])
        low = int((lb <= tau * (1 - 1e-4)).sum()) - 4
        high = int((lb <= tau * (1 + 1e-3) + 1e-6).sum())
        assert low <= s["leaves_initial"] <= high, (j, low, s["leaves_initial"], high)


@pytest.mark.parametrize("length,w", [(128, 16), (200, 8)])
def test_hybrid_other_lengths_and_sorted_rows(isax, length, w):
    # other filter row classes (len_pad 128 and 256 with padding) and the leaf-order FP32 rows
    X = workload.random_walks(30_011, length, seed=71 + length, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 60, seed=72)
    Q = torch.cat([Qn, workload.fresh_queries(20, length, seed=73, device="cuda")]).contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Q), 5)
    for prec in (1, 5):
        idx = isax.Index(X, w, 8, leaf_size=64, precision=prec)
        for limit in (1, 20, 10**6):
            ids, d, st = idx.query(Q, k=5, mode="hybrid", hybrid_leaves=limit, stats=True)
            _check(ids, d, ref_ids, ref_d2, 5)
            li = np.array([s["leaves_initial"] for s in st])
            path = np.array([s["path"] for s in st])
            assert np.all(path[li <= limit] == isax.MODE_INDEX)
        idx.close()


@pytest.mark.parametrize("k", [1, 10, 100])
def test_hybrid_cost_model_routes(isax, coll, k):
    # the planner's own routes at 100K series, without a limit and without the batch
    # shortcut: its plain choice; the filter priced at 1000x (the plain index path after
    # the sampled pre-screen) and at 1/1000 (the pre-screen sends the queries to the filter,
    # which start from their approximate answers).  Every route gives the oracle's answer.
    idx, Q, X = coll["idx"], coll["Q"], coll["X"]
    ref_ids, ref_d2 = (coll["ids"], coll["d2"]) if k <= 10 else kr.knn_exact_c(_cpu(X), _cpu(Q), k)
    ib, db = idx.query(Q, k=k, mode="bf16")
    paths = {}
    for extra in (0, isax.QF_FILTER_DEAR, isax.QF_FILTER_CHEAP):
        ids, d, st = idx.query(Q, k=k, mode="hybrid", flags=isax.QF_NO_SHORTCUT | extra, stats=True)
        _check(ids, d, ref_ids, ref_d2, k)
        paths[extra] = {s["path"] for s in st}
        assert torch.equal(ids, ib) and torch.equal(d.view(torch.int32), db.view(torch.int32))
    assert paths[isax.QF_FILTER_DEAR] == {isax.MODE_INDEX}
    assert paths[isax.QF_FILTER_CHEAP] == {isax.MODE_BF16}
