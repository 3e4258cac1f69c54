"""Parity at the benchmark's full size: 100M x 256 random walks, 1000 noisy
queries per batch (the launch configuration bench.py times), every mode.

The oracle cannot scan 100M series for every query, so a sample of queries
(twenty per noise level, sixty in all) is checked: their exact answers come
from the C oracle streamed over the whole collection in 10M-series chunks.
For every other query each returned distance is checked with the oracle one
pair at a time, and the ordering of the row.
"""
import os
import sys

import numpy as np
import pytest
import torch

import workload
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu

N = int(os.environ.get("ISAX_FULLSIZE_N", 100_000_000))
M = 1000


def say(*a):
    print("[fullsize]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < N * 256 * 4 * 1.9:
        pytest.skip("not enough device memory for the full-size collection")
    import paper_2009_01614_amd as isax
    say("generating", N, "x 256")
    X = workload.random_walks(N, 256, seed=20090163, device="cuda")
    Q, src, sig = workload.noisy_queries(X, M, seed=20091163)
    say("building")
    idx = isax.Index(X, 16, 8, precision=3)
    sample = np.concatenate([np.where(sig == s)[0][:20] for s in (0.01, 0.1, 1.0)])
    say("oracle over", N, "series for queries", sample.tolist())
    st = kr.KnnState(Q[sample].cpu().numpy(), 10)
    CH = 10_000_000
    for a in range(0, N, CH):
        st.merge(X[a:a + CH].cpu().numpy(), a)
    say("oracle done")
    yield {"isax": isax, "X": X, "Q": Q, "idx": idx, "sample": sample, "ids": st.ids, "d2": st.d2}
    idx.close()


@pytest.mark.parametrize("mode", ["index", "scan", "bf16", "fp8", "hybrid"])
@pytest.mark.parametrize("k", [1, 10])
def test_fullsize_sampled_parity(big, mode, k):
    say("query", mode, "k =", k)
    ids, d = big["idx"].query(big["Q"], k=k, mode=mode)
    s = big["sample"]
    got_ids = ids[s].cpu().numpy()
    assert np.array_equal(got_ids, big["ids"][:, :k])
    ref = np.sqrt(big["d2"][:, :k])
    assert np.all(np.abs(d[s].cpu().numpy() - ref) <= 1e-4 * ref)
    # every returned distance of the whole batch, oracle pair by pair
    X, Q = big["X"], big["Q"]
    rows = X[ids[:, :k].reshape(-1)].cpu().numpy().reshape(M, k, -1)
    Qh = Q.cpu().numpy()
    d2 = np.stack([kr.sq_dists(rows[i], Qh[i]) for i in range(M)])
    dd = d.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dd - np.sqrt(d2)) <= 1e-4 * np.sqrt(d2))
    assert np.all(np.diff(dd, axis=1) >= 0)
