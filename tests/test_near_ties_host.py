"""The near-tie inputs are what they claim to be (CPU only).

For every planted case the FP64 oracle must order the tied series by their
exact distances (higher id first), while the FP32 sums of the FP32 differences
rank them equal (kind "equal") or the lower id first (kind "inverted") in
every summation order tried; so a final ordering without a compensated
recompute returns the wrong ids on these inputs (checked with a plain FP32
brute force).  The GPU tests then run the same construction.
"""
import numpy as np

import workload
from oracle import knn_ref as kr
from tests import near_ties as nt


def _cases():
    X = workload.random_walks(20_003, 256, seed=20090167).numpy()
    Q, cases = nt.plant_cases(X, seed=20091167)
    return X, Q, cases


def test_construction_properties():
    X, Q, cases = _cases()
    for c in cases:
        q = Q[c["query"]]
        ids = c["ids"]
        d64 = [nt.d2_exact(q, X[i]) for i in ids]
        f32 = [nt.fp32_sums(q, X[i]) for i in ids]
        for j in range(1, len(ids)):
            assert ids[j] > ids[j - 1]
            # exact: the higher id is closer, by far more than FP64 or Dot2 rounding
            assert d64[j] < d64[j - 1] and (d64[j - 1] - d64[j]) / d64[j] > 1e-10, (c, d64)
            if c["kind"] == "equal":
                assert f32[j] == f32[0], (c, f32)
                diff_a = np.float32(q) - X[ids[0]]
                diff_b = np.float32(q) - X[ids[j]]
                assert np.array_equal(diff_a.astype(np.float32), diff_b.astype(np.float32))
            else:
                assert all(b >= a for a, b in zip(f32[0], f32[j])), (c, f32)
                assert f32[j][0] > f32[0][0]


def test_oracle_orders_by_exact_distance_and_fp32_rule_does_not():
    X, Q, cases = _cases()
    kmax = 12
    ref_ids, ref_d2 = kr.knn_exact(X, Q, kmax)
    for c in cases:
        r = ref_ids[c["query"]]
        m = len(c["closer"])
        tied = c["ids"]
        assert sorted(r[:m].tolist()) == sorted(c["closer"]), (c, r)
        assert r[m:m + len(tied)].tolist() == tied[::-1], (c, r)
    # a plain FP32 scan ordered by (FP32 value, id) gets these cases wrong
    d = (Q[:, None, :].astype(np.float32) - X[None, :, :]).astype(np.float32)
    d32 = np.einsum("mnt,mnt->mn", d, d, dtype=np.float32)
    for c in cases:
        j = c["query"]
        order = np.lexsort((np.arange(X.shape[0]), d32[j]))[:kmax]
        assert not np.array_equal(order, ref_ids[j]), c
