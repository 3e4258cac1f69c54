"""Near-tie planting for the tests of the final ordering (test infrastructure).

A near tie is a pair of series x_a (lower id) and x_b (higher id) whose exact
distances to a query q order b first, while every FP32 computation that starts
from the FP32 differences fl(q_t - x_t) ranks them equal, or a first.  The
plain FP32 rule (value, then lower id) therefore returns a; the oracle, and a
correct tie guard, return b (Sec. II, Similarity Search, with ties broken by the
lower id; the order itself is decided by the exact distances).

Construction, all in FP32 values checked with exact FP64 arithmetic:
  - "equal": at every coordinate x_b moves towards q_t by as many ulps as keep
    fl(q_t - x_b,t) == fl(q_t - x_a,t).  The FP32 differences are then the same
    numbers, so any FP32 sum of their squares, in any order, is the same; the
    exact distance of b is smaller.
  - "inverted": as "equal", and one coordinate t2 (where q_t2 = 3.3, most of
    the distance) is set so that q_t2 - x_a,t2 lies just below a rounding
    midpoint and q_t2 - x_b,t2 just above it: fl(q - x_b) is one ulp larger,
    so every FP32 sum for b is >= the one for a (FP32 addition and fma are
    monotone) and the sequential one is larger, while the exact distances
    differ at t2 by about 1e-14 only, far less than the gain of the others.
This module holds no part of the search method: it only plants inputs.
"""
from __future__ import annotations

import numpy as np


def _step(x: np.float32, toward: float, s: int) -> np.float32:
    """x moved s ulps towards `toward` (no sign change: s is capped by the caller)."""
    v = np.array([x], np.float32)
    b = v.view(np.int32)[0]
    up = (toward > float(x)) == (float(x) >= 0)   # moving away from zero increases |bits|
    nb = b + s if up else b - s
    return np.array([nb], np.int32).view(np.float32)[0]


def _max_equal_steps(q: np.float32, x: np.float32) -> int:
    """Largest s with fl(q - x') == fl(q - x) for x' = x moved s ulps towards q."""
    d0 = np.float32(q - x)
    if float(q) == float(x):
        return 0

    def ok(s):
        xs = _step(x, float(q), s)
        if np.sign(xs) != np.sign(x) and float(x) != 0.0:
            return False
        # must stay on the same side of q
        if (float(q) - float(xs)) * (float(q) - float(x)) <= 0:
            return False
        return np.float32(q - xs) == d0

    lo, hi = 0, 1
    while hi < (1 << 30) and ok(hi):
        lo, hi = hi, hi * 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo


def nudge_equal(q: np.ndarray, xa: np.ndarray, frac: float = 1.0) -> np.ndarray:
    """x_b with fl32(q - x_b) == fl32(q - x_a) everywhere and a smaller exact distance."""
    xb = xa.copy()
    for t in range(xa.shape[0]):
        s = int(_max_equal_steps(q[t], xa[t]) * frac)
        if s > 0:
            xb[t] = _step(xa[t], float(q[t]), s)
    return xb


def set_midpoint_coordinate(q: np.ndarray, xa: np.ndarray, xb: np.ndarray, t2: int):
    """Rewrites coordinate t2 of x_a and x_b (q_t2 must be in (0.5, 4)): q - x_a rounds down, q - x_b up."""
    Q2 = float(q[t2])
    assert 0.5 < Q2 < 4.0
    e = np.floor(np.log2(Q2))
    h = 2.0 ** (e - 24)                     # half an ulp of q_t2
    xa[t2] = np.float32(-h)
    xa[t2] = _step(_step(xa[t2], 0.0, 1), 0.0, 1)        # -(h - 2 ulp): q - x_a below the midpoint
    xb[t2] = np.float32(-h)
    xb[t2] = _step(_step(xb[t2], -1.0, 1), -1.0, 1)      # -(h + 2 ulp): q - x_b above it
    assert np.float32(q[t2] - xa[t2]) == np.float32(Q2)
    assert np.float32(q[t2] - xb[t2]) > np.float32(Q2)


def d2_exact(q: np.ndarray, x: np.ndarray) -> float:
    d = q.astype(np.float64) - x.astype(np.float64)
    return float(np.sum(d * d))


def fp32_sums(q: np.ndarray, x: np.ndarray) -> list:
    """FP32 sums of squared FP32 differences in three orders: sequential fma-free, pairwise, 16-lane."""
    d = (q.astype(np.float32) - x.astype(np.float32)).astype(np.float32)
    sq = (d * d).astype(np.float32)
    seq = np.float32(0)
    for v in sq:
        seq = np.float32(seq + v)
    pair = np.float32(np.sum(sq, dtype=np.float32))
    lanes = np.zeros(16, np.float32)
    for t in range(0, d.shape[0], 4):
        g = (t // 4) % 16
        for e in range(4):
            if t + e < d.shape[0]:
                lanes[g] = np.float32(lanes[g] + sq[t + e])
    while lanes.shape[0] > 1:
        h = lanes.shape[0] // 2
        lanes = (lanes[:h] + lanes[h:]).astype(np.float32)
    return [float(seq), float(pair), float(lanes[0])]


def plant_cases(X: np.ndarray, seed: int):
    """Plants the near-tie cases into X (FP32 [n, len], modified in place).

    Returns (queries FP32 [m, len], list of case dicts).  Each case: query row,
    the tied ids (ascending id, exact distances descending), the kind, and the
    number of planted series that are closer than the tie.
    """
    n, L = X.shape
    rng = np.random.default_rng(seed)
    specs = [("equal", 0, 2), ("inverted", 0, 2), ("equal", 9, 2), ("inverted", 9, 2), ("equal", 1, 2),
             ("equal", 0, 3), ("inverted", 1, 2)]
    used = set()

    def fresh_id(lo, hi):
        while True:
            i = int(rng.integers(lo, hi))
            if i not in used:
                used.add(i)
                return i

    Q, cases = [], []
    for kind, closer, chain in specs:
        a = fresh_id(0, n // 2)
        base = X[a].astype(np.float64)
        q = (base + rng.standard_normal(L) * 0.1).astype(np.float32)
        if kind == "inverted":
            # the midpoint coordinate carries most of the distance, so that its
            # one-ulp excess in FP32 survives the rounding of the sum
            t2 = int(np.argmax(q))
            q[t2] = np.float32(3.3)
        xa = X[a].copy()
        rows = [xa]
        for j in range(1, chain):
            rows.append(nudge_equal(q, xa, frac=j / (chain - 1)))
        if kind == "inverted":
            for j in range(1, chain):
                set_midpoint_coordinate(q, rows[0], rows[j], t2)
        ids = [a] + sorted(fresh_id(n // 2, n) for _ in range(chain - 1))
        for i, r in zip(ids, rows):
            X[i] = r
        near = []
        for _ in range(closer):
            c = fresh_id(0, n)
            X[c] = (q.astype(np.float64) + rng.standard_normal(L) * 0.03).astype(np.float32)
            near.append(c)
        Q.append(q)
        cases.append({"kind": kind, "ids": ids, "closer": near, "query": len(Q) - 1})
    return np.stack(Q), cases
