"""Pins of the DTW oracle (oracle/dtw_ref.py and its C twin) against what the
definition and the mathematics fix: a hand-worked example, brute-force path
enumeration, the no-warping special case, symmetry, monotonicity in the band,
and the chain of lower bounds the index prunes with."""
import os

import numpy as np
import pytest

from oracle import dtw_ref as dr
from oracle import isax_ref as ir
from oracle import knn_ref as kr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dtw_example.txt")


def _rng(seed):
    return np.random.default_rng(seed)


def _walks(rng, n, L):
    X = np.cumsum(rng.standard_normal((n, L)), axis=1)
    X = (X - X.mean(1, keepdims=True)) / X.std(1, keepdims=True)
    return X.astype(np.float32)


def test_hand_worked_example():
    rows = [ln for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 5
    for ln in rows:
        qs, xs, rs, vs = (p.strip() for p in ln.split(";"))
        q = np.array(qs.split(), np.float32)
        x = np.array(xs.split(), np.float32)
        r, v = int(rs), float(vs)
        assert dr.dtw_sq(x[None, :], q, r)[0] == v
        assert kr.dtw_sq_c(x[None, :], q, r)[0] == v
        assert dr.dtw_sq_paths(q, x, r) == v


@pytest.mark.parametrize("L", [1, 2, 3, 5, 6])
def test_recurrence_equals_path_enumeration(L):
    rng = _rng(L)
    for trial in range(4):
        q = rng.standard_normal(L).astype(np.float32)
        x = rng.standard_normal(L).astype(np.float32)
        for r in range(L):
            ref = dr.dtw_sq_paths(q, x, r)
            got = dr.dtw_sq(x[None, :], q, r)[0]
            assert abs(got - ref) <= 1e-12 * max(ref, 1e-300), (L, r, got, ref)


def test_no_warping_is_squared_euclidean():
    rng = _rng(1)
    X = _walks(rng, 50, 40)
    q = _walks(rng, 1, 40)[0]
    assert np.array_equal(dr.dtw_sq(X, q, 0), kr.sq_dists(X, q))


def test_symmetry_and_band_monotone():
    rng = _rng(2)
    X = _walks(rng, 20, 48)
    q = _walks(rng, 1, 48)[0]
    prev = None
    for r in (0, 1, 2, 5, 12, 47):
        a = dr.dtw_sq(X, q, r)
        b = np.array([dr.dtw_sq(q[None, :], x, r)[0] for x in X])
        assert np.array_equal(a, b)
        if prev is not None:
            assert np.all(a <= prev)
        prev = a


def test_c_twin_bit_identical_and_knn():
    rng = _rng(3)
    X = _walks(rng, 3000, 64)
    Q = _walks(rng, 5, 64)
    for r in (0, 6, 20):
        ids, d2 = dr.knn_dtw(X[:400], Q[:2], 7, r)
        ids_c, d2_c = kr.knn_dtw_c(X[:400], Q[:2], 7, r)
        assert np.array_equal(ids, ids_c) and np.array_equal(d2, d2_c)
    # no warping: the same neighbours as the Euclidean oracle
    ids0, d0 = kr.knn_dtw_c(X, Q, 10, 0)
    ide, de = kr.knn_exact_c(X, Q, 10)
    assert np.array_equal(ids0, ide) and np.array_equal(d0, de)
    # streaming in chunks gives the same lists
    st = kr.KnnState(Q, 10, 6)
    st.merge(X[:1234], 0)
    st.merge(X[1234:], 1234)
    ids6, d6 = kr.knn_dtw_c(X, Q, 10, 6)
    assert np.array_equal(st.ids, ids6) and np.array_equal(st.d2, d6)


def test_envelope():
    rng = _rng(4)
    q = rng.standard_normal(30).astype(np.float32)
    U, L = dr.envelope(q, 0)
    assert np.array_equal(U, q) and np.array_equal(L, q)
    U, L = dr.envelope(q, 3)
    assert np.all(U >= q) and np.all(L <= q)
    assert U[10] == q[7:14].max() and L[0] == q[:4].min()


@pytest.mark.parametrize("r", [0, 4, 16])
def test_lower_bound_chain(r):
    """iSAX envelope bound <= LB_Keogh <= DTW^2, and for r = 0 LB_Keogh = ED^2."""
    rng = _rng(5 + r)
    X = _walks(rng, 400, 128)
    Q = np.concatenate([_walks(rng, 3, 128), X[:2] + 0.1 * rng.standard_normal((2, 128)).astype(np.float32)])
    words = ir.isax_words(X, 16, 8)
    for q in Q:
        d = dr.dtw_sq(X, q, r)
        lk = dr.lb_keogh_sq(X, q, r)
        li = dr.isax_envelope_bound_sq(q, words, 8, 16, r)
        assert np.all(lk <= d * (1 + 1e-12))
        assert np.all(li <= lk * (1 + 1e-12) + 1e-12)
        if r == 0:
            assert np.allclose(lk, kr.sq_dists(X, q), rtol=1e-12)
            assert np.allclose(li, ir.mindist_sq(ir.paa64(q[None, :], 16)[0], words, ir.breakpoints(8), 8),
                               rtol=1e-12)
    # the bounds are not vacuous on near-duplicate queries
    assert np.mean(lk > 0) > 0.5
