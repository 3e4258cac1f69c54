"""Pins for the CPU oracle: closed forms, library routines, invariants and brute force.

Each test would fail on a plausible mistake in the oracle (dropped term,
wrong sign or index, transposed operand, off-by-one region).
"""
import itertools
import math
import os

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

from oracle import isax_ref as ir
from oracle import knn_ref as kr
from oracle import margin_ref as mr
from oracle import spectral_ref as sr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def walks(n, length, seed):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.standard_normal((n, length)), axis=1)
    return ((t - t.mean(1, keepdims=True)) / t.std(1, keepdims=True)).astype(np.float32)


# ----------------------------------------------------------------------------- PAA
def test_paa_ramp_closed_form():
    X = np.arange(256, dtype=np.float32)[None, :]
    want = 16 * np.arange(16) + 7.5
    assert np.array_equal(ir.paa64(X, 16)[0], want)
    assert np.array_equal(ir.paa32_tree(X, 16)[0], want.astype(np.float32))


def test_paa_constant_and_linearity():
    X = walks(50, 128, 1)
    c = np.full((3, 128), 2.25, np.float32)
    assert np.all(ir.paa64(c, 16) == 2.25) and np.all(ir.paa32_tree(c, 16) == 2.25)
    a, b = 3.0, -1.5
    lhs = ir.paa64(a * X.astype(np.float64) + b, 16)
    assert np.allclose(lhs, a * ir.paa64(X, 16) + b, rtol=0, atol=1e-12)


def test_paa_brute_force_tiny():
    X = walks(4, 24, 2)
    for w in (1, 2, 3, 4, 6, 8, 12, 24):
        m = 24 // w
        got = ir.paa64(X, w)
        for i in range(4):
            for j in range(w):
                exact = math.fsum(float(v) for v in X[i, j * m:(j + 1) * m]) / m
                assert abs(got[i, j] - exact) <= 4e-16 * max(1.0, abs(exact))


def test_paa32_tree_order_and_error_bound():
    # non-power-of-two segment: zero padding must not change an exact integer sum
    X = np.arange(12, dtype=np.float32)[None, :]
    assert np.array_equal(ir.paa32_tree(X, 4)[0], np.array([1, 4, 7, 10], np.float32))
    # explicit tree for m = 4: ((x0 + x1) + (x2 + x3)) / 4 in FP32
    Y = walks(200, 64, 3)
    a = Y.reshape(200, 16, 4)
    want = ((a[:, :, 0] + a[:, :, 1]) + (a[:, :, 2] + a[:, :, 3])) / np.float32(4)
    assert np.array_equal(ir.paa32_tree(Y, 16), want)
    # any-order FP32 mean of m terms is within m * 2^-23 * max|x| of the FP64 mean
    Z = walks(500, 256, 4)
    err = np.abs(ir.paa32_tree(Z, 16).astype(np.float64) - ir.paa64(Z, 16))
    assert err.max() <= 16 * 2.0 ** -23 * np.abs(Z).max()


# ----------------------------------------------------------------------------- breakpoints
def _golden_quantiles():
    out = {}
    with open(os.path.join(GOLDEN, "normal_quantiles.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c, *vals = line.split()
            out[int(c)] = np.array([float(v) for v in vals])
    return out


def test_breakpoints_golden_table():
    for c, vals in _golden_quantiles().items():
        assert np.allclose(ir.breakpoints(c), vals, atol=5e-5)


def test_breakpoints_against_erf_cdf():
    # Phi(beta_j) = j / 2^c, with Phi from the stdlib error function
    for c in range(1, 9):
        beta = ir.breakpoints(c)
        assert len(beta) == 2 ** c - 1
        phi = np.array([0.5 * (1 + math.erf(b / math.sqrt(2))) for b in beta])
        assert np.allclose(phi, np.arange(1, 2 ** c) / 2 ** c, rtol=0, atol=1e-13)
        assert np.all(np.diff(beta) > 0)
        assert np.allclose(beta, -beta[::-1], atol=1e-14)          # symmetry
        assert beta[2 ** (c - 1) - 1] == 0.0                       # median edge is exactly 0


def test_breakpoints_nest_across_cardinalities():
    for c in range(2, 9):
        fine = ir.breakpoints_f32(c)
        for b in range(1, c):
            coarse = ir.breakpoints_f32(b)
            step = 2 ** (c - b)
            assert np.array_equal(coarse, fine[step - 1::step])


def test_c8_table_span():
    beta = ir.breakpoints(8)
    assert abs(beta[-1] - 2.6601) < 1e-4 and abs(beta[0] + 2.6601) < 1e-4
    assert abs(np.diff(beta).min() - 0.00979) < 1e-5


# ----------------------------------------------------------------------------- empirical edges
def _embeddings(n, d, seed):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((40, d)) * 3.0
    return (centres[rng.integers(0, 40, n)] + 0.7 * rng.standard_normal((n, d))).astype(np.float32)


def test_empirical_edges_are_inverted_cdf_quantiles():
    # edge j is the library's inverted-CDF quantile of the sampled segment means at j / 2^c
    X = _embeddings(3000, 64, 21)
    for c in (1, 3, 8):
        got = ir.empirical_breakpoints(X, 8, c)
        v = ir.paa32_tree(X, 8).ravel()   # n < 65536 / 8: every series is sampled
        want = np.quantile(v, np.arange(1, 2 ** c) / 2 ** c, method="inverted_cdf")
        assert got.dtype == np.float32 and np.array_equal(got, want.astype(np.float32))


def test_empirical_edges_rank_property_brute_force():
    # #{v < e_j} < ceil(j V / 2^c) <= #{v <= e_j}, counted one value at a time
    X = _embeddings(500, 24, 22)
    v = [float(a) for a in ir.paa32_tree(X, 6).ravel()]
    V = len(v)
    for c in (2, 4):
        e = ir.empirical_breakpoints(X, 6, c)
        assert np.all(np.diff(e) >= 0)
        for j in range(1, 2 ** c):
            rank = -(-j * V // 2 ** c)
            below = sum(1 for a in v if a < e[j - 1])
            upto = sum(1 for a in v if a <= e[j - 1])
            assert below < rank <= upto


def test_empirical_edges_sample_rule_and_nesting():
    # series i holds the constant i, so the sampled values name the sampled series:
    # S = ceil(65536 / w) series, series floor(t n / S); nesting across cardinalities
    n, w = 50_000, 8
    X = np.repeat(np.arange(n, dtype=np.float32)[:, None], 32, axis=1)
    S = 8192
    picked = sorted({t * n // S for t in range(S)})
    assert len(picked) == S
    e8 = ir.empirical_breakpoints(X, w, 8)
    assert set(e8.astype(np.int64)) <= set(picked)
    for j in range(1, 256):                       # each series contributes w equal values
        assert e8[j - 1] == picked[-(-j * S // 256) - 1]
    for b in range(1, 8):
        step = 2 ** (8 - b)
        assert np.array_equal(ir.empirical_breakpoints(X, w, b), e8[step - 1::step])


def test_empirical_edges_approach_normal_quantiles_and_skip_nan():
    # piecewise-constant N(0,1) segments: the sampled means are the normal draws themselves,
    # so the edges approach Phi^-1(j / 16) (DKW: |F_V - Phi| < 0.01 with V = 65536)
    rng = np.random.default_rng(23)
    seg = rng.standard_normal((8192, 8)).astype(np.float32)
    X = np.repeat(seg, 16, axis=1)
    e = ir.empirical_breakpoints(X, 8, 4)
    assert np.array_equal(ir.paa32_tree(X, 8), seg)
    phi = np.array([0.5 * (1 + math.erf(float(b) / math.sqrt(2))) for b in e])
    assert np.abs(phi - np.arange(1, 16) / 16).max() < 0.01
    # a series with a non-finite value: its segment means are dropped before the ranks
    Y = X.copy()
    Y[5, 3] = np.nan
    keep = np.isfinite(ir.paa32_tree(Y, 8).ravel())
    assert keep.sum() == Y.size // 16 - 1
    v = np.sort(ir.paa32_tree(Y, 8).ravel()[keep])
    j = np.arange(1, 16)
    assert np.array_equal(ir.empirical_breakpoints(Y, 8, 4), v[-(-(j * v.size) // 16) - 1])


def test_isax_words_with_explicit_edges():
    X = _embeddings(200, 32, 24)
    assert np.array_equal(ir.isax_words(X, 8, 4, ir.breakpoints_f32(4)), ir.isax_words(X, 8, 4))
    e = ir.empirical_breakpoints(X, 8, 4)
    got = ir.isax_words(X, 8, 4, e)
    p = ir.paa32_tree(X, 8)
    for i in range(0, 200, 37):
        for j in range(8):
            assert got[i, j] == sum(1 for b in e if b <= p[i, j])
    # the empirical edges spread the symbols: each of the 16 regions holds about 1/16
    h = np.bincount(got.ravel(), minlength=16) / got.size
    assert h.min() > 0.04 and h.max() < 0.09


# ----------------------------------------------------------------------------- symbols
def test_symbols_brute_force_and_half_open():
    beta = ir.breakpoints_f32(3)
    vals = np.concatenate([beta, np.nextafter(beta, -np.inf), np.nextafter(beta, np.inf),
                           np.float32([-9, 9, 0])]).astype(np.float32)
    got = ir.symbols(vals, beta)
    for v, s in zip(vals, got):
        assert s == sum(1 for b in beta if b <= v)
    # a value exactly on beta_j belongs to region j (the region above)
    assert np.array_equal(ir.symbols(beta, beta), np.arange(1, 8))


def test_symbols_prefix_property_and_msb():
    X = walks(300, 256, 5)
    p = ir.paa32_tree(X, 16)
    s8 = ir.symbols(p, ir.breakpoints_f32(8))
    for b in range(1, 8):
        assert np.array_equal(s8 >> (8 - b), ir.symbols(p, ir.breakpoints_f32(b)))
    assert np.array_equal(s8 >> 7, (p >= 0).astype(np.uint8))


def test_symbols_uniform_on_normal_samples():
    rng = np.random.default_rng(6)
    v = rng.standard_normal(256 * 400).astype(np.float32)
    h = np.bincount(ir.symbols(v, ir.breakpoints_f32(8)), minlength=256)
    exp = len(v) / 256
    chi2 = ((h - exp) ** 2 / exp).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


def test_paper_word_example():
    with open(os.path.join(GOLDEN, "isax_word_example.txt")) as f:
        row = [l for l in f if not l.startswith("#")][0].split()
    w, c = int(row[0]), int(row[1])
    word = np.array([[int(s) for s in row[3].split(",")]], np.uint8)
    assert ir.word_string(word[0], c) == row[2].replace("_", " ")
    assert ir.root_subtree(word, c)[0] == int(row[4].replace(",", ""), 2)
    bits = ir.interleaved_bits(word, c)[0]
    assert "".join(str(int(b)) for b in bits) == row[5]
    assert ir.key_prefix(word, c)[0] == np.uint64(int(row[5], 2) << (64 - w * c))


def test_interleaved_key_brute_force():
    rng = np.random.default_rng(7)
    words = rng.integers(0, 256, size=(40, 16), dtype=np.uint8)
    keys = ir.key_prefix(words, 8, 64)
    for i in range(40):
        s = "".join(format(int(words[i, j]), "08b")[r] for r in range(8) for j in range(16))
        assert int(keys[i]) == int(s[:64], 2)
        assert ir.root_subtree(words[i:i + 1], 8)[0] == int(s[:16], 2)


def test_sorted_order_and_envelopes():
    X = walks(3000, 256, 8)
    words = ir.isax_words(X, 16, 8)
    order = ir.sorted_order(words, 8, 64)
    assert np.array_equal(np.sort(order), np.arange(3000))
    keys = ir.key_prefix(words, 8, 64)[order]
    assert np.all(keys[1:] >= keys[:-1])
    ties = keys[1:] == keys[:-1]
    assert np.all(order[1:][ties] > order[:-1][ties])
    lo, hi = ir.leaf_envelopes(words[order], 256)
    assert lo.shape == (12, 16)
    for leaf in range(12):
        blk = words[order[leaf * 256:(leaf + 1) * 256]]
        assert np.all(blk >= lo[leaf]) and np.all(blk <= hi[leaf])
        assert np.all(blk.min(0) == lo[leaf]) and np.all(blk.max(0) == hi[leaf])


# ----------------------------------------------------------------------------- mindist
def _ed2(q, X):
    return ((X.astype(np.float64) - q.astype(np.float64)) ** 2).sum(axis=1)


@pytest.mark.parametrize("kind", ["random", "noisy", "self"])
def test_mindist_lower_bounds_distance(kind):
    X = walks(2000, 256, 9)
    rng = np.random.default_rng(10)
    beta = ir.breakpoints(8)
    words = ir.symbols(ir.paa64(X, 16), beta)
    for t in range(10):
        if kind == "random":
            q = walks(1, 256, 100 + t)[0]
        elif kind == "noisy":
            q = X[rng.integers(2000)] + rng.normal(0, [0.01, 0.1, 1][t % 3], 256).astype(np.float32)
        else:
            q = X[t]
        lb = ir.mindist_sq(ir.paa64(q[None], 16)[0], words, beta, 16)
        assert np.all(lb <= _ed2(q, X) * (1 + 1e-12))
        if kind == "self":
            assert lb[t] == 0.0


def test_mindist_tight_case_and_brute_force():
    beta = ir.breakpoints(3)
    m, w = 4, 3
    p = np.array([-2.0, 0.1, 1.5])                   # query segment means
    xs = np.array([beta[0], beta[3], beta[5]])       # series values exactly on region lower edges
    s = ir.symbols(xs, beta)                         # regions 1, 4, 6
    assert list(s) == [1, 4, 6]
    q = np.repeat(p, m)[None, :]
    x = np.repeat(xs, m)[None, :]
    lb = ir.mindist_sq(p, s[None, :], beta, m)[0]
    # segment 0: p below region 1 -> distance beta_1 - p = |x - p|; segment 1: p=0.1 is below
    # region 4 = [0, 0.3186): p inside -> 0; segment 2: p=1.5 above region 6 = [0.6745, 1.1503)
    ext = np.concatenate([[-np.inf], beta, [np.inf]])
    want = m * ((ext[1] - p[0]) ** 2 + 0.0 + (p[2] - ext[7]) ** 2)
    assert abs(lb - want) <= 1e-12
    # where the query is on the far side of the region edge the bound is tight
    assert abs(m * (ext[1] - p[0]) ** 2 - ((q[0, :4] - x[0, :4]) ** 2).sum()) <= 1e-12


def test_mindist_monotone_in_cardinality_and_envelope():
    X = walks(1500, 256, 11)
    q = walks(1, 256, 12)[0]
    pq = ir.paa64(q[None], 16)[0]
    prev = None
    for c in range(1, 9):
        beta = ir.breakpoints(c)
        lb = ir.mindist_sq(pq, ir.symbols(ir.paa64(X, 16), beta), beta, 16)
        if prev is not None:
            assert np.all(lb >= prev - 1e-12)
        prev = lb
    beta = ir.breakpoints(8)
    words = ir.symbols(ir.paa64(X, 16), beta)
    lo, hi = ir.leaf_envelopes(words, 100)
    elb = ir.envelope_mindist_sq(pq, lo, hi, beta, 16)
    for leaf in range(len(lo)):
        assert np.all(elb[leaf] <= prev[leaf * 100:(leaf + 1) * 100] + 1e-12)


def test_mindist_pure_python_tiny():
    beta = ir.breakpoints(2)
    ext = [-math.inf] + list(beta) + [math.inf]
    rng = np.random.default_rng(13)
    words = rng.integers(0, 4, size=(20, 4))
    p = rng.normal(size=4)
    got = ir.mindist_sq(p, words, beta, 8)
    for i in range(20):
        tot = 0.0
        for j in range(4):
            s = words[i, j]
            d = max(0.0, ext[s] - p[j], p[j] - ext[s + 1])
            tot += d * d
        assert abs(got[i] - 8 * tot) <= 1e-12 * max(1, tot)


# ----------------------------------------------------------------------------- spectral copy
def test_dct_matrix_cosine_definition_and_orthonormal():
    # scipy's DCT against the cosine definition, term by term (pure Python), and T T^T = I
    L = 12
    T = sr.dct_matrix(L)
    for i in range(L):
        c = math.sqrt((1.0 if i == 0 else 2.0) / L)
        for j in range(L):
            k = i * (2 * j + 1) % (4 * L)   # cos has period 4L in units of pi / (2L)
            assert abs(T[i, j] - c * math.cos(math.pi * k / (2 * L))) <= 1e-15
    for L in (16, 200, 256, 512):
        T = sr.dct_matrix(L)
        assert np.abs(T @ T.T - np.eye(L)).max() <= 1e-13


def test_spectral_ext_pure_python_tiny():
    X = walks(5, 8, 40)
    got = sr.spectral_ext(X, 3)
    for i in range(5):
        y = [math.fsum((math.sqrt((1.0 if k == 0 else 2.0) / 8) * math.cos(math.pi * (k * (2 * j + 1) % 32) / 16)) *
                       float(X[i, j]) for j in range(8)) for k in range(8)]
        want = [y[0], y[1], math.sqrt(math.fsum(v * v for v in y[2:]))]
        assert np.allclose(got[i], want, rtol=0, atol=1e-13)


def test_spectral_ext_energy_bound_and_monotone_in_width():
    X = walks(300, 256, 41)
    Q = walks(20, 256, 42)
    d2 = np.stack([kr.sq_dists(X, q) for q in Q])
    assert np.allclose(np.linalg.norm(sr.spectral_ext(X, 128), axis=1), np.linalg.norm(X.astype(np.float64), axis=1),
                       rtol=1e-13, atol=0)
    prev = None
    for D in (2, 16, 64, 127, 128, 192, 256):
        lb = sr.spectral_lb_sq(Q, X, D)
        assert np.all(lb <= d2 * (1 + 1e-12) + 1e-9), D        # a lower bound on every pair
        if prev is not None:
            assert np.all(lb >= prev * (1 - 1e-12) - 1e-9), D  # never weaker with more coefficients
        prev = lb
    # D = L keeps every coefficient but the sign of the last: exact where the signs agree
    Y, Z = sr.spectral_ext(Q, 256), sr.spectral_ext(X, 256)
    from scipy.fft import dct
    same = np.sign(dct(Q.astype(np.float64), norm="ortho", axis=1)[:, -1:]) == \
        np.sign(dct(X.astype(np.float64), norm="ortho", axis=1)[:, -1])[None, :]
    assert np.allclose(np.where(same, prev, d2), d2, rtol=1e-10, atol=1e-9)


def test_spectral_ext_tight_case():
    # q = x + v with v in the span of the first D - 1 basis vectors: equal tails, so LB = ED^2
    X = walks(50, 256, 43)
    T = sr.dct_matrix(256)
    rng = np.random.default_rng(44)
    V = rng.standard_normal((50, 127)) @ T[:127]
    Q = X.astype(np.float64) + V
    lb = np.array([sr.spectral_lb_sq(Q[i:i + 1], X[i:i + 1], 128)[0, 0] for i in range(50)])
    assert np.allclose(lb, (V ** 2).sum(axis=1), rtol=1e-10, atol=0)


def test_spectral_filter_scores_bound_every_pair():
    # the filter's approximate distance minus its error bound never exceeds ED^2 (FP64),
    # and the bound is far tighter on random walks than the BF16 margin on the full rows is wide
    X = walks(2000, 256, 45)
    rng = np.random.default_rng(46)
    src = rng.integers(0, 2000, 30)
    Q = X[src] + np.array([0.01, 0.1, 1.0])[np.arange(30) % 3, None] * rng.standard_normal((30, 256))
    Q = ((Q - Q.mean(1, keepdims=True)) / Q.std(1, keepdims=True)).astype(np.float32)
    approx, err = sr.spectral_filter_scores(Q, X, 128)
    d2 = np.stack([kr.sq_dists(X, q) for q in Q])
    assert np.all(approx - err <= d2 + 1e-9)
    lb = sr.spectral_lb_sq(Q, X, 128)
    assert np.all(np.abs(lb - approx) <= err + 1e-9)
    assert err.mean() < 4.0
    # a planted mistake: dropping the tail coordinate breaks the bound somewhere
    e_q, e_x = sr.spectral_ext(Q, 128), sr.spectral_ext(X, 128)
    no_tail = (e_q[:, None, :127] - e_x[None, :, :127]) ** 2
    assert np.all(no_tail.sum(axis=2) <= d2 + 1e-9)
    wrong = (Q.astype(np.float64) ** 2).sum(1)[:, None] + (X.astype(np.float64) ** 2).sum(1)[None, :] - \
        2.0 * (e_q[:, :127] @ e_x[:, :127].T)
    assert np.any(wrong > d2 + 1e-6)


# ----------------------------------------------------------------------------- k-NN
def test_knn_pure_python_brute_force():
    X = walks(60, 16, 14)
    Q = walks(5, 16, 15)
    ids, d2 = kr.knn_exact(X, Q, 7)
    for j in range(5):
        D = [math.fsum((float(Q[j, t]) - float(X[i, t])) ** 2 for t in range(16)) for i in range(60)]
        want = sorted(range(60), key=lambda i: (D[i], i))[:7]
        assert list(ids[j]) == want
        assert np.allclose(d2[j], [D[i] for i in want], rtol=1e-14, atol=0)


def test_knn_against_scipy_cdist():
    X = walks(3000, 128, 16)
    Q = walks(8, 128, 17)
    ids, d2 = kr.knn_exact(X, Q, 10)
    ref = cdist(Q.astype(np.float64), X.astype(np.float64), "sqeuclidean")
    for j in range(8):
        assert np.array_equal(ids[j], np.argsort(ref[j], kind="stable")[:10])
        assert np.allclose(d2[j], ref[j][ids[j]], rtol=1e-13)


def test_knn_duplicates_self_query_and_prefix():
    X = walks(500, 64, 18)
    X[300] = X[17]
    X[401] = X[17]
    ids, d2 = kr.knn_exact(X, X[[17, 300, 42]], 5)
    assert list(ids[0][:3]) == [17, 300, 401] and list(ids[1][:3]) == [17, 300, 401]
    assert np.all(d2[:2, :3] == 0.0)
    assert ids[2][0] == 42 and d2[2][0] == 0.0
    ids1, d21 = kr.knn_exact(X, X[[17, 300, 42]], 1)
    assert np.array_equal(ids1[:, 0], ids[:, 0]) and np.array_equal(d21[:, 0], d2[:, 0])


def test_knn_c_twin_bit_exact_and_chunked():
    X = walks(4000, 256, 19)
    Q = walks(6, 256, 20)
    X[3999] = X[5]
    Q[1] = X[5]
    ids, d2 = kr.knn_exact(X, Q, 10)
    ids_c, d2_c = kr.knn_exact_c(X, Q, 10)
    assert np.array_equal(ids, ids_c) and np.array_equal(d2, d2_c)
    st = kr.KnnState(Q, 10)
    for a in range(0, 4000, 1500):
        st.merge(X[a:a + 1500], a)
    assert np.array_equal(st.ids, ids) and np.array_equal(st.d2, d2)
    assert np.array_equal(kr.sq_dists_c(X, Q[0]), kr.sq_dists(X, Q[0]))


# ----------------------------------------------------------------------------- quantisers / margin
def test_bf16_round_matches_torch():
    rng = np.random.default_rng(21)
    x = (rng.standard_normal(100000) * rng.choice([1e-3, 1, 30], 100000)).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mr.bf16_round(x), want)


def test_e4m3_round_matches_torch():
    rng = np.random.default_rng(22)
    X = walks(400, 256, 23) * np.float32(3)
    xt, s = mr.quantise_rows(X, "fp8")
    assert np.all(np.abs(X).max(1) / s <= 448) and np.all(np.abs(X).max(1) / (s / 2) > 448)
    y = (X.astype(np.float64) / s[:, None]).astype(np.float32)
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy() * s[:, None]
    assert np.array_equal(xt, want)
    v = (rng.standard_normal(50000) * 0.02).astype(np.float32)   # includes the subnormal range
    want_v = torch.from_numpy(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(mr.e4m3_round(v.astype(np.float64)), want_v)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_dot_error_bound_holds(kind):
    X = walks(300, 256, 24)
    Q = walks(20, 256, 25)
    xt, _ = mr.quantise_rows(X, kind)
    qt, _ = mr.quantise_rows(Q, kind)
    err = np.abs(Q.astype(np.float64) @ X.astype(np.float64).T - qt @ xt.T)
    bound = mr.dot_error_bound(Q, X, qt, xt)
    assert np.all(err <= bound * (1 + 1e-12))
    assert bound.mean() > 10 * err.mean() or kind == "bf16"


def test_oracle_brute_force_itertools_tiny():
    # every pair of rows, distances by itertools, matches the ordered answer at k = n
    X = walks(9, 8, 26)
    q = walks(1, 8, 27)
    ids, d2 = kr.knn_exact(X, q, 9)
    pairs = sorted((sum((float(a) - float(b)) ** 2 for a, b in zip(q[0], X[i])), i)
                   for i in itertools.islice(range(9), 9))
    assert [i for _, i in pairs] == list(ids[0])
