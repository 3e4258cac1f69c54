"""Serving loop: continuous batching, results identical alone and in the mix."""
import threading
import time

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


@pytest.fixture(scope="module")
def colls(isax):
    A = workload.random_walks(60_001, 256, seed=20090165, device="cuda")
    B = workload.random_walks(30_001, 128, seed=20090166, device="cuda")
    return [A, B]


def _requests(colls, n_req, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        c = int(rng.integers(2))
        X = colls[c]
        k = int(rng.choice([1, 10, 100]))
        if rng.random() < 0.2:
            q = workload.fresh_queries(1, X.shape[1], seed=seed * 1000 + i, device="cuda")[0]
        else:
            q, _, _ = workload.noisy_queries(X, 1, seed=seed * 1000 + i, sigmas=(float(rng.choice([0.01, 0.1, 1.0])),))
            q = q[0]
        reqs.append((c, q.cpu().numpy(), k))
    return reqs


def _serve(isax, indexes, reqs, mode="index", rate_hz=2000.0, **opt):
    srv = isax.Server(indexes, mode=mode, **opt)
    out = {}
    rng = np.random.default_rng(5)

    def producer():
        # a burst (arrivals while the first batches run), then Poisson arrivals
        for tag, (c, q, k) in enumerate(reqs):
            srv.submit(c, q, k, tag)
            if tag >= len(reqs) // 3:
                time.sleep(rng.exponential(1.0 / rate_hz))

    th = threading.Thread(target=producer)
    th.start()
    deadline = time.time() + 120
    while len(out) < len(reqs) and time.time() < deadline:
        for r in srv.poll(50):
            out[r["tag"]] = r
    th.join()
    srv.close()
    assert len(out) == len(reqs)
    return out


def _overlapping(out):
    """Two requests taken in at different times whose service intervals overlap."""
    iv = sorted((r["t_start"], r["t_done"]) for r in out.values())
    return any(iv[i + 1][0] > iv[i][0] and iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))


# (mode, server options): batch-level admission, and step-level admission (the
# filter modes' default) with small tables so that rows are reused
CASES = [("index", dict(max_batch=16, streams=3)), ("hybrid", dict(max_batch=16, streams=3)),
         ("bf16", dict(max_batch=16, streams=3, batches=True)), ("bf16", dict(max_batch=24, chunks=8)),
         ("fp8", dict(max_batch=24, chunks=5)), ("bf16", dict(max_batch=7, chunks=1))]


@pytest.mark.parametrize("mode,opt", CASES, ids=[f"{m}-{'-'.join(f'{k}{v}' for k, v in o.items())}" for m, o in CASES])
def test_alone_equals_mix_and_oracle(isax, colls, mode, opt):
    indexes = [isax.Index(X, 16, 8, precision={"bf16": 1, "hybrid": 1, "fp8": 2}.get(mode, 0)) for X in colls]
    reqs = _requests(colls, 90, seed=11)
    out = _serve(isax, indexes, reqs, mode=mode, **opt)
    Xh = [X.cpu().numpy() for X in colls]
    sizes = set()
    for tag, (c, q, k) in enumerate(reqs):
        r = out[tag]
        assert r["status"] == 0, r["message"]
        sizes.add(r["batch_size"])
        qt = torch.from_numpy(q[None]).cuda()
        ids1, d1 = indexes[c].query(qt, k=k, mode=mode)
        assert r["ids"] == ids1[0].tolist()
        assert np.array_equal(np.array(r["dists"], np.float32), d1[0].cpu().numpy())  # bit-identical
        ref_ids, ref_d2 = kr.knn_exact_c(Xh[c], q[None], k)
        assert r["ids"] == ref_ids[0].tolist()
        assert np.allclose(r["dists"], np.sqrt(ref_d2[0]), rtol=1e-4, atol=0)
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
    assert max(sizes) > 1, "no request was served together with another"
    assert _overlapping(out), "no two requests taken in at different times were in service together"


def test_step_level_rows_that_need_a_run_of_their_own(isax, colls):
    # 3000 copies of one series: a query equal to it ties with all of them, more than the
    # table's final ordering takes, so the engine answers it by itself; the others are unaffected
    X = colls[0].clone()
    rng = np.random.default_rng(20091173)
    dup = np.sort(rng.choice(X.shape[0], size=3000, replace=False))
    X[torch.as_tensor(dup[1:], device="cuda")] = X[int(dup[0])].clone()
    idx = isax.Index(X, 16, 8, precision=1)
    reqs = [(0, X[int(dup[0])].cpu().numpy(), 5)] + [(0, q, k) for c, q, k in _requests([X, colls[1]], 40, seed=13)
                                                      if c == 0]
    out = _serve(isax, [idx], reqs, mode="bf16", max_batch=16, chunks=4)
    r = out[0]
    assert r["status"] == 0 and r["ids"] == dup[:5].tolist() and r["dists"] == [0.0] * 5
    Xh = X.cpu().numpy()
    for tag, (c, q, k) in enumerate(reqs):
        ref_ids, _ = kr.knn_exact_c(Xh, q[None], k)
        assert out[tag]["ids"] == ref_ids[0].tolist()


def test_memory_budget_forces_small_batches(isax, colls):
    indexes = [isax.Index(X, 16, 8) for X in colls]
    reqs = _requests(colls, 30, seed=12)
    out = _serve(isax, indexes, reqs, max_batch=64, streams=2, memory_budget=1)
    for tag, (c, q, k) in enumerate(reqs):
        assert out[tag]["status"] == 0 and out[tag]["batch_size"] == 1
