"""Exact k-NN under dynamic time warping in FP64, and its lower bounds (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

The paper names DTW as the second common distance of similarity search
(Sec. II, Similarity Search) and states that the same index answers DTW
queries without change (Sec. V).  It does not write DTW out; this module
uses the usual definition with a Sakoe-Chiba band of half-width r:

  D(i, j) = (q_i - x_j)^2 + min(D(i-1, j-1), D(i-1, j), D(i, j-1)),
            for |i - j| <= r, D(-1, -1) = 0, every other cell outside the
            band or the grid = +inf;
  DTW_r(q, x)^2 = D(len-1, len-1),

every cell computed in FP64 from the FP32 inputs as d = q_i - x_j (exact),
d * d (rounded), then + min (rounded); the minimum is exact, so every cell
has one value whatever order the grid is filled in.  The answer is the first
k series ordered by (DTW^2, id), distance sqrt(DTW^2).

Lower bounds (used by the method for pruning, checked here as invariants):
  envelope(q, r):  U_i = max q[i-r .. i+r],  L_i = min q[i-r .. i+r]
  LB_Keogh^2 = sum_i (x_i - U_i)^2 [x_i > U_i] + (L_i - x_i)^2 [x_i < L_i]
  iSAX bound^2 = m * sum_j max(0, beta_lo(s_j) - PAA(U)_j, PAA(L)_j - beta_hi(s_j))^2
with iSAX bound <= LB_Keogh <= DTW_r^2 (the second by Keogh's envelope
argument, the first by Cauchy-Schwarz per segment and because the PAA of x
lies in the region of its symbol).
"""
from __future__ import annotations

import numpy as np

from . import isax_ref as ir


def dtw_sq(X: np.ndarray, q: np.ndarray, r: int) -> np.ndarray:
    """DTW_r(q, x)^2 of one query against every row of X, FP64, by the recurrence."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float32))
    n, L = X.shape
    q64 = np.asarray(q, dtype=np.float32).astype(np.float64)
    X64 = X.astype(np.float64)
    inf = np.full(n, np.inf)
    prev = np.full((n, L), np.inf)       # row i-1 of D over j
    for i in range(L):
        cur = np.full((n, L), np.inf)
        for j in range(max(0, i - r), min(L, i + r + 1)):
            d = q64[i] - X64[:, j]
            c = d * d
            if i == 0 and j == 0:
                m = np.zeros(n)
            else:
                diag = prev[:, j - 1] if (i > 0 and j > 0) else inf
                up = prev[:, j] if i > 0 else inf
                left = cur[:, j - 1] if j > 0 else inf
                m = np.minimum(np.minimum(diag, up), left)
            cur[:, j] = c + m
        prev = cur
    return prev[:, L - 1]


def dtw_sq_paths(q, x, r: int) -> float:
    """DTW_r^2 by enumerating every warping path (tiny inputs only), summed exactly."""
    import math
    q = [float(v) for v in np.asarray(q, np.float32)]
    x = [float(v) for v in np.asarray(x, np.float32)]
    L = len(q)
    best = math.inf

    def walk(i, j, terms):
        nonlocal best
        terms = terms + [(q[i] - x[j]) ** 2]
        if i == L - 1 and j == L - 1:
            best = min(best, math.fsum(terms))
            return
        for di, dj in ((1, 1), (1, 0), (0, 1)):
            a, b = i + di, j + dj
            if a < L and b < L and abs(a - b) <= r:
                walk(a, b, terms)

    walk(0, 0, [])
    return best


def knn_dtw(X: np.ndarray, Q: np.ndarray, k: int, r: int):
    """Exact k-NN under DTW_r: (ids int64 [m, k], squared distances float64 [m, k])."""
    X = np.asarray(X, dtype=np.float32)
    Q = np.asarray(Q, dtype=np.float32).reshape(-1, X.shape[1])
    n = X.shape[0]
    if not 1 <= k <= n:
        raise ValueError("k must be in 1..n")
    ids = np.empty((Q.shape[0], k), np.int64)
    d2 = np.empty((Q.shape[0], k), np.float64)
    all_ids = np.arange(n, dtype=np.int64)
    for j, q in enumerate(Q):
        D = dtw_sq(X, q, r)
        order = np.lexsort((all_ids, D))[:k]
        ids[j] = order
        d2[j] = D[order]
    return ids, d2


def envelope(q: np.ndarray, r: int):
    """(U, L): running max and min of q over the window [i - r, i + r], FP32 values."""
    q = np.asarray(q, dtype=np.float32)
    L = q.shape[0]
    U = np.array([q[max(0, i - r):min(L, i + r + 1)].max() for i in range(L)], np.float32)
    Lo = np.array([q[max(0, i - r):min(L, i + r + 1)].min() for i in range(L)], np.float32)
    return U, Lo


def lb_keogh_sq(X: np.ndarray, q: np.ndarray, r: int) -> np.ndarray:
    """LB_Keogh^2 of every row of X against the envelope of q, FP64."""
    U, Lo = envelope(q, r)
    X64 = np.atleast_2d(np.asarray(X, np.float32)).astype(np.float64)
    above = np.maximum(0.0, X64 - U.astype(np.float64))
    below = np.maximum(0.0, Lo.astype(np.float64) - X64)
    return (above * above + below * below).sum(axis=1)


def isax_envelope_bound_sq(q: np.ndarray, words: np.ndarray, c: int, w: int, r: int) -> np.ndarray:
    """iSAX lower bound of DTW_r^2: the PAA of the query envelope against every word's regions, FP64."""
    U, Lo = envelope(q, r)
    pu = ir.paa64(U[None, :], w)[0]
    pl = ir.paa64(Lo[None, :], w)[0]
    m = ir.segment_length(U.shape[0], w)
    beta = ir.breakpoints(c)
    lower = np.concatenate([[-np.inf], beta])
    upper = np.concatenate([beta, [np.inf]])
    words = np.asarray(words, dtype=np.int64)
    d = np.maximum(0.0, np.maximum(lower[words] - pu[None, :], pl[None, :] - upper[words]))
    return m * (d * d).sum(axis=1)
