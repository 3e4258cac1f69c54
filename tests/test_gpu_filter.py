"""Reduced-precision filter: FP64 check of the error margin on every pair, and exact answers.

The margin M returned for each (query, series) pair must satisfy
|ED^2_FP64 - approx| <= M, where approx = |q|^2 + |x|^2 - 2 q~.x~ is what the
matrix cores computed; the answers through the filter must equal the oracle's.
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


def _cpu(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
@pytest.mark.parametrize("length", [256, 128, 200])
def test_margin_bounds_fp64_error_on_every_pair(isax, mode, length):
    X = workload.random_walks(12_007, length, seed=31 + length, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 30, seed=32)
    Q = torch.cat([Qn, workload.fresh_queries(10, length, seed=33, device="cuda")]).contiguous()
    idx = isax.Index(X, 16 if length % 16 == 0 else 8, 8, precision=3)
    approx, margin = (_cpu(t).astype(np.float64) for t in idx.filter_scores(Q, mode))
    Xh, Qh = _cpu(X), _cpu(Q)
    worst = 0.0
    for j in range(Q.shape[0]):
        d2 = kr.sq_dists(Xh, Qh[j])
        err = np.abs(d2 - approx[j])
        assert np.all(err <= margin[j]), (j, (err - margin[j]).max())
        worst = max(worst, (err / margin[j]).max())
    assert margin.mean() < (8.0 if mode == "bf16" else 80.0) * length / 256
    print(f"{mode} len {length}: mean margin {margin.mean():.3f}, worst err/margin {worst:.3f}")


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
@pytest.mark.parametrize("k", [1, 10])
def test_filter_answers_match_oracle(isax, mode, k):
    X = workload.random_walks(100_003, 256, seed=20090162, device="cuda")
    workload.planted_duplicates(X, [(99_000, 5)])
    Qn, _, _ = workload.noisy_queries(X, 21, seed=20091164)
    Q = torch.cat([Qn, workload.fresh_queries(5, 256, seed=7, device="cuda"), X[5:6].clone()]).contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Q), k)
    idx = isax.Index(X, 16, 8, precision=3)
    ids, d = idx.query(Q, k=k, mode=mode)
    assert np.array_equal(_cpu(ids), ref_ids)
    ref = np.sqrt(ref_d2)
    err = np.abs(_cpu(d) - ref) / np.maximum(ref, 1e-30)
    err[ref == 0] = np.abs(_cpu(d)[ref == 0])
    assert err.max() <= 1e-4


def test_filter_many_query_tiles_and_ragged(isax):
    X = workload.random_walks(30_001, 128, seed=41, device="cuda")
    Q = workload.fresh_queries(700, 128, seed=42, device="cuda")
    ref_ids, _ = kr.knn_exact_c(_cpu(X), _cpu(Q), 3)
    idx = isax.Index(X, 16, 8, precision=3)
    for mode in ("bf16", "fp8"):
        ids, _ = idx.query(Q, k=3, mode=mode)
        assert np.array_equal(_cpu(ids), ref_ids)


@pytest.mark.parametrize("mode", ["bf16", "fp8"])
def test_filter_candidate_overflow_path(isax, mode):
    X = workload.random_walks(50_021, 256, seed=51, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 40, seed=52)
    Q = torch.cat([Qn, workload.fresh_queries(8, 256, seed=53, device="cuda")]).contiguous()
    ref_ids, _ = kr.knn_exact_c(_cpu(X), _cpu(Q), 10)
    idx = isax.Index(X, 16, 8, precision=3)
    for cap in (16, 200):
        ids, _ = idx.query(Q, k=10, mode=mode, candidate_capacity=cap)
        assert np.array_equal(_cpu(ids), ref_ids), cap


@pytest.mark.parametrize("m", [64, 65, 100, 128, 129, 200, 256, 257])
def test_filter_batch_size_classes(isax, m):
    """Every block configuration (64, 128, 256, 512 queries per block) and its boundaries."""
    X = workload.random_walks(40_009, 256, seed=61, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, m, seed=62 + m)
    ref_ids, _ = kr.knn_exact_c(_cpu(X), _cpu(Qn), 3)
    idx = isax.Index(X, 16, 8, precision=3)
    for mode in ("bf16", "fp8"):
        ids, _ = idx.query(Qn.contiguous(), k=3, mode=mode)
        assert np.array_equal(_cpu(ids), ref_ids), mode


@pytest.mark.parametrize("length,m", [(128, 200), (200, 129), (250, 256), (64, 150)])
def test_filter_256_row_class_other_lengths(isax, length, m):
    # 129-256 queries take eight-wave blocks of 256 rows: other row lengths (len_pad 64, 128, 256)
    # and lengths that are not a multiple of 4
    X = workload.random_walks(25_013, length, seed=81 + length, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, m, seed=82 + m)
    ref_ids, ref_d2 = kr.knn_exact_c(_cpu(X), _cpu(Qn), 4)
    w = 16 if length % 16 == 0 else (10 if length % 10 == 0 else 2)
    idx = isax.Index(X, w, 8, precision=3)
    for mode in ("bf16", "fp8", "hybrid"):
        kw = dict(hybrid_leaves=3) if mode == "hybrid" else {}
        ids, d = idx.query(Qn.contiguous(), k=4, mode=mode, **kw)
        assert np.array_equal(_cpu(ids), ref_ids), mode
        ref = np.sqrt(ref_d2)
        err = np.abs(_cpu(d) - ref) / np.maximum(ref, 1e-30)
        err[ref == 0] = np.abs(_cpu(d)[ref == 0])
        assert err.max() <= 1e-4, mode
