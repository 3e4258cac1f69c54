"""Spectral copy of the BF16 filter: the leading DCT-II coefficients of every
series plus the norm of the rest, in BF16.

* The filter's scores on that copy satisfy approx - M <= ED^2 (FP64) on every
  pair, and approx is within M of the oracle's spectral lower bound.
* Answers through the filter (BF16 and hybrid modes, the server) equal the
  oracle's: ids bit for bit, distances within 1e-4 relative, and equal the
  full-length copy's answers bit for bit.
"""
import time

import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr
from oracle import spectral_ref as sr

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


def _check(ids, d, ref_ids, ref_d2, k):
    ids, d = _cpu(ids), _cpu(d)
    assert np.array_equal(ids, ref_ids[:, :k])
    ref = np.sqrt(ref_d2[:, :k])
    err = np.abs(d.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    err[ref == 0] = np.abs(d[ref == 0])
    assert err.max() <= RTOL, err.max()


def _default_dim(length):
    lp = (length + 63) // 64 * 64
    return min(256, max(64, lp * 3 // 4 // 64 * 64))


@pytest.mark.parametrize("length,dim", [(256, 0), (256, 64), (256, 128), (128, 0), (200, 0), (384, 0), (512, 0)])
def test_spectral_scores_bound_every_pair(isax, length, dim):
    X = workload.random_walks(6_007, length, seed=71 + length, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 30, seed=72)
    Q = torch.cat([Qn, workload.fresh_queries(10, length, seed=73, device="cuda")]).contiguous()
    w = 16 if length % 16 == 0 else 8
    idx = isax.Index(X, w, 8, precision=isax.PREC_SPECTRAL, spectral_dim=dim)
    D = dim or _default_dim(length)
    assert idx.info()["spectral_dim"] == D and idx.info()["has_bf16"] == 0
    approx, margin = (_cpu(t).astype(np.float64) for t in idx.filter_scores(Q, "bf16"))
    Xh, Qh = _cpu(X), _cpu(Q)
    lb = sr.spectral_lb_sq(Qh, Xh, D)
    for j in range(Q.shape[0]):
        d2 = kr.sq_dists(Xh, Qh[j])
        assert np.all(approx[j] - margin[j] <= d2), (j, (approx[j] - margin[j] - d2).max())
        assert np.all(np.abs(lb[j] - approx[j]) <= margin[j]), (j, (np.abs(lb[j] - approx[j]) - margin[j]).max())
    assert margin.mean() < 8.0 * length / 256


@pytest.fixture(scope="module")
def coll(isax):
    X = workload.random_walks(100_003, 256, seed=20090171, device="cuda")
    workload.planted_duplicates(X, [(99_998, 21), (40_000, 21)])
    Qn, _, sig = workload.noisy_queries(X, 150, seed=20091171)
    Q = torch.cat([Qn, workload.fresh_queries(6, 256, seed=20091172, device="cuda"), X[21:22].clone()]).contiguous()
    both = isax.Index(X, 16, 8, precision=isax.PREC_BF16 | isax.PREC_SPECTRAL)
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Q), 100)
    return {"X": X, "Q": Q, "idx": both, "ids": ref_ids, "d2": ref_d2, "sig": sig}


@pytest.mark.parametrize("k", [1, 10, 100])
@pytest.mark.parametrize("mode", ["bf16", "hybrid"])
def test_spectral_answers_match_oracle(isax, coll, mode, k):
    idx, Q = coll["idx"], coll["Q"]
    ids, d = idx.query(Q, k=k, mode=mode)
    _check(ids, d, coll["ids"], coll["d2"], k)
    # the full-length copy gives the same bits
    ids2, d2 = idx.query(Q, k=k, mode=mode, flags=isax.QF_FULL_ROWS)
    assert torch.equal(ids, ids2) and torch.equal(d, d2)


@pytest.mark.parametrize("route", ["cheap", "dear", "split"])
def test_spectral_hybrid_routes(isax, coll, route):
    idx, Q = coll["idx"], coll["Q"]
    flags = isax.QF_NO_SHORTCUT | {"cheap": isax.QF_FILTER_CHEAP, "dear": isax.QF_FILTER_DEAR, "split": 0}[route]
    # split: queries with more than one leaf left after the first round take the filter
    kw = {"hybrid_leaves": 1} if route == "split" else {}
    ids, d, st = idx.query(Q, k=10, mode="hybrid", flags=flags, stats=True, **kw)
    _check(ids, d, coll["ids"], coll["d2"], 10)
    paths = [s["path"] for s in st]
    if route == "cheap":
        assert set(paths) == {isax.MODES["bf16"]}
    if route == "dear":
        assert set(paths) == {isax.MODES["index"]}
    if route == "split":
        assert paths.count(isax.MODES["bf16"]) > 0


def test_spectral_small_batches_and_per_query_k(isax, coll):
    idx, Q = coll["idx"], coll["Q"]
    kq = torch.tensor([1 + (i * 7) % 50 for i in range(Q.shape[0])], dtype=torch.int32, device="cuda")
    ids, d = idx.query(Q, k=50, mode="bf16", k_per_query=kq, batch=37)
    ids, d = _cpu(ids), _cpu(d)
    for i in range(Q.shape[0]):
        k = int(kq[i])
        assert np.array_equal(ids[i, :k], coll["ids"][i, :k])
        assert np.all(ids[i, k:] == -1)
    # the 64-query block class and one query alone
    for m in (1, 64):
        ids, d = idx.query(Q[:m].contiguous(), k=10, mode="bf16")
        _check(ids, d, coll["ids"][:m], coll["d2"][:m], 10)


def test_spectral_only_index_and_errors(isax, coll):
    X, Q = coll["X"], coll["Q"]
    idx = isax.Index(X, 16, 8, precision=isax.PREC_SPECTRAL)
    ids, d = idx.query(Q, k=10, mode="hybrid")
    _check(ids, d, coll["ids"], coll["d2"], 10)
    with pytest.raises(isax.IsaxError):
        idx.query(Q, k=10, mode="bf16", flags=isax.QF_FULL_ROWS)
    for bad in (32, 96, 256, 320):
        with pytest.raises(isax.IsaxError):
            isax.Index(X, 16, 8, precision=isax.PREC_SPECTRAL, spectral_dim=bad)
    with pytest.raises(isax.IsaxError):
        isax.Index(X, 16, 8, precision=isax.PREC_BF16, spectral_dim=128)
    short = workload.random_walks(1000, 64, seed=5, device="cuda")
    with pytest.raises(isax.IsaxError):
        isax.Index(short, 16, 8, precision=isax.PREC_SPECTRAL)


def test_spectral_noalloc_and_server(isax, coll):
    idx, Q = coll["idx"], coll["Q"]
    a = idx.query(Q, k=10, mode="hybrid")
    b = idx.query(Q, k=10, mode="hybrid", noalloc=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # step-level server over the spectral copy
    X = coll["X"]
    only = isax.Index(X, 16, 8, precision=isax.PREC_SPECTRAL)
    srv = isax.Server([only], mode="bf16", chunks=4)
    try:
        Qh = _cpu(Q)
        for i in range(Q.shape[0]):
            srv.submit(0, Qh[i], 10, tag=i)
        got = {}
        t_end = time.time() + 60
        while len(got) < Q.shape[0] and time.time() < t_end:
            for r in srv.poll(1000):
                got[r["tag"]] = r
        assert len(got) == Q.shape[0]
    finally:
        srv.close()
    for i, r in got.items():
        assert r["status"] == 0, r
        assert np.array_equal(np.asarray(r["ids"]), coll["ids"][i, :10])


def test_spectral_switch_to_full_rows(isax, coll):
    # with both copies the filter decides after a second sample of the collection: far
    # queries at k = 100 switch the rest of the pass to the full rows, near queries at
    # k = 1 stay on the spectral copy; the answers are the oracle's either way
    idx, Q, sig = coll["idx"], coll["Q"], coll["sig"]
    cases = [("far", np.where(sig == 1.0)[0], 100, True), ("near", np.where(sig == 0.01)[0], 1, False)]
    for name, rows, k, want in cases:
        sel = torch.from_numpy(rows).cuda()
        isax.profile_reset()
        isax.profile_enable(True)
        try:
            ids, d = idx.query(Q[sel].contiguous(), k=k, mode="bf16")
            prof = isax.profile_read()
        finally:
            isax.profile_enable(False)
        assert ("filter_full_rows_switch" in prof) == want, (name, sorted(prof))
        _check(ids, d, coll["ids"][rows], coll["d2"][rows], k)
