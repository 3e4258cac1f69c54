"""DTW at the size its measurement runs: 10M x 256 random walks, window 25,
100 noisy queries in one batch, index and plain-scan modes, FP32 rows in leaf
order (the launch configuration bench.py --next-report times).

The oracle cannot run DTW against 10M series for every query, so: one query's
exact answer from the C oracle over the whole collection; every returned
distance of the batch recomputed by the oracle pair by pair; and for ten
queries, no series of a random sample of 20,000 lies closer than the k-th
answer (a property that holds at any size)."""
import os
import sys

import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu

N = int(os.environ.get("ISAX_DTW_FULLSIZE_N", 10_000_000))
M, R, K = 100, 25, 10


def say(*a):
    print("[fullsize-dtw]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    say("generating", N, "x 256")
    X = workload.random_walks(N, 256, seed=20090165, device="cuda")
    Q, src, sig = workload.noisy_queries(X, M, seed=20091165)
    idx = isax.Index(X, 16, 8, precision=4)
    out = {}
    for mode in ("index", "scan"):
        say("query", mode)
        out[mode] = idx.query(Q, k=K, mode=mode, metric="dtw", window=R)
    Xh = X.cpu().numpy()
    yield {"X": X, "Xh": Xh, "Q": Q, "Qh": Q.cpu().numpy(), "sig": sig, "out": out}
    idx.close()


def test_dtw_modes_agree(big):
    assert torch.equal(big["out"]["index"][0], big["out"]["scan"][0])
    assert torch.equal(big["out"]["index"][1], big["out"]["scan"][1])


def test_dtw_one_query_exact(big):
    j = int(np.where(big["sig"] == 0.1)[0][0])
    say("oracle over", N, "series for query", j)
    ids, d2 = kr.knn_dtw_c(big["Xh"], big["Qh"][j:j + 1], K, R)
    got_ids, got_d = (t[j].cpu().numpy() for t in big["out"]["index"])
    assert np.array_equal(got_ids, ids[0])
    assert np.all(np.abs(got_d - np.sqrt(d2[0])) <= 1e-4 * np.sqrt(d2[0]))


def test_dtw_returned_distances_and_sampled_property(big):
    ids, d = (t.cpu().numpy() for t in big["out"]["index"])
    Xh, Qh = big["Xh"], big["Qh"]
    for i in range(M):
        ref = kr.dtw_sq_c(Xh[ids[i]], Qh[i], R)
        assert np.all(np.abs(d[i].astype(np.float64) - np.sqrt(ref)) <= 1e-4 * np.sqrt(ref)), i
    assert np.all(np.diff(d, axis=1) >= 0)
    rng = np.random.default_rng(7)
    sample = rng.choice(N, 20_000, replace=False)
    for i in range(0, M, 10):
        dd = kr.dtw_sq_c(Xh[sample], Qh[i], R)
        kth = np.float64(d[i, -1]) ** 2
        closer = sample[dd < kth * (1 - 1e-5)]
        assert np.all(np.isin(closer, ids[i])), (i, closer[:5])
