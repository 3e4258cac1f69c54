"""iSAX summarisation and lower bounds, written out plainly (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Paper: "Data Series Indexing Gone Parallel" (Peng, Fatourou, Palpanas).
  * PAA: each series is cut into w segments of equal length and every
    segment is replaced by the mean of its points (Sec. II, iSAX
    Representation).
  * iSAX: the value axis is cut into regions, each region has a bit-string
    symbol, and a segment takes the symbol of the region its mean falls in
    (Sec. II, iSAX Representation).  The paper does not state the region
    edges; we use the standard-normal quantiles Phi^-1(j / 2^c), j=1..2^c-1,
    with half-open regions [beta_s, beta_{s+1}) and s = 0 the lowest region.
  * Root subtree of a series = the first bit of each of its w symbols
    (Sec. III, ParIS/ParIS+ approach); cardinality refinement appends one bit
    to one segment (Sec. II, ADS+ Index).  Our flat layout orders series by
    the bit-interleaved key (first bits of all segments, then second bits, ...)
    and cuts the order into fixed-size leaves with per-segment symbol
    envelopes.
  * Lower bound: the distance between the query's raw values (through its
    PAA) and a series' iSAX summary (Sec. III, MESSI approach); we use the
    iSAX MINDIST of the work cited there for the representation.

Precision: FP64 unless a function says otherwise.  The symbol of a segment is
a quantised code decided by floating point, so `paa32_tree` computes the
segment mean in FP32 in one fixed order (zero-pad the segment to a power of
two, add adjacent pairs level by level, divide by the segment length) and
`isax_words` compares it with the FP32-rounded breakpoints: that is the
precision the GPU kernel decides in.
"""
from __future__ import annotations

import numpy as np
from scipy.stats import norm


def segment_length(length: int, w: int) -> int:
    """Points per segment; segments have equal length (Sec. II, iSAX Representation)."""
    if w < 1 or length < 1 or length % w:
        raise ValueError(f"length {length} is not a multiple of segments {w}")
    return length // w


def paa64(X: np.ndarray, w: int) -> np.ndarray:
    """Segment means in FP64: paa[i, j] = mean of X[i, j*m:(j+1)*m] (Sec. II)."""
    X = np.asarray(X)
    n, length = X.shape
    m = segment_length(length, w)
    return X.astype(np.float64).reshape(n, w, m).sum(axis=2) / m


def paa32_tree(X: np.ndarray, w: int) -> np.ndarray:
    """Segment means in FP32 with one fixed summation order.

    The segment is zero-padded to the next power of two, adjacent pairs are
    added level by level (a balanced binary tree over contiguous halves), and
    the total is divided by the true segment length m in FP32.
    """
    X = np.asarray(X, dtype=np.float32)
    n, length = X.shape
    m = segment_length(length, w)
    p = 1
    while p < m:
        p *= 2
    a = X.reshape(n, w, m)
    if p != m:
        a = np.concatenate([a, np.zeros((n, w, p - m), np.float32)], axis=2)
    while a.shape[2] > 1:
        a = a[:, :, 0::2] + a[:, :, 1::2]
    return a[:, :, 0] / np.float32(m)


def breakpoints(c: int) -> np.ndarray:
    """beta_j = Phi^-1(j / 2^c), j = 1..2^c-1, ascending, FP64."""
    if not 1 <= c <= 8:
        raise ValueError("card_bits must be in 1..8")
    return norm.ppf(np.arange(1, 2 ** c, dtype=np.float64) / 2.0 ** c)


def breakpoints_f32(c: int) -> np.ndarray:
    """The FP64 breakpoints rounded to nearest FP32."""
    return breakpoints(c).astype(np.float32)


EDGE_SAMPLE = 65536  # segment means the empirical edges are taken from (about)


def empirical_breakpoints(X: np.ndarray, w: int, c: int) -> np.ndarray:
    """Region edges from the collection's own segment means (data that is not
    z-normalised, e.g. the embedding vectors of Sec. V), FP32, ascending.

    Sample: the FP32 segment means (paa32_tree) of every segment of
    S = min(n, ceil(EDGE_SAMPLE / w)) series, series floor(t n / S) for t < S;
    V = S w values.  Edge j (j = 1..2^c-1) is the ceil(j V / 2^c)-th smallest
    of them: the smallest value whose empirical CDF reaches j / 2^c.
    """
    X = np.asarray(X, dtype=np.float32)
    n = X.shape[0]
    S = min(n, -(-EDGE_SAMPLE // w))
    rows = (np.arange(S, dtype=np.int64) * n) // S
    v = paa32_tree(X[rows], w).ravel()
    v = np.sort(v[np.isfinite(v)])
    V = v.shape[0]
    j = np.arange(1, 2 ** c, dtype=np.int64)
    return v[-(-(j * V) // 2 ** c) - 1].astype(np.float32)


def symbols(paa: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Region index s = #{j : beta_j <= paa} (half-open regions, s=0 lowest)."""
    return np.searchsorted(beta, paa, side="right").astype(np.uint8)


def isax_words(X: np.ndarray, w: int, c: int, beta: np.ndarray | None = None) -> np.ndarray:
    """uint8 [n, w]: the c-bit iSAX symbol of every segment of every series
    (region edges beta, FP32; default the standard-normal ones)."""
    return symbols(paa32_tree(X, w), breakpoints_f32(c) if beta is None else beta)


def word_string(word, c: int) -> str:
    """Bit-string form of a word, e.g. symbols (2, 0, 3) at c=2 -> '10 00 11'."""
    return " ".join(format(int(s), f"0{c}b") for s in word)


def interleaved_bits(words: np.ndarray, c: int) -> np.ndarray:
    """bool [n, w*c]: bit r of every segment in turn, most significant bit first.

    Position r*w + j holds bit (c-1-r) of segment j, so the first w positions
    are the root-subtree id (first bit of each segment) and every further
    block of w positions refines every segment by one bit.
    """
    words = np.asarray(words, dtype=np.uint8)
    n, w = words.shape
    out = np.zeros((n, w * c), dtype=bool)
    for r in range(c):
        for j in range(w):
            out[:, r * w + j] = (words[:, j] >> (c - 1 - r)) & 1
    return out


def key_prefix(words: np.ndarray, c: int, nbits: int = 64) -> np.ndarray:
    """uint64: the first min(nbits, w*c) interleaved bits, left-aligned (bit 63 first)."""
    bits = interleaved_bits(words, c)
    nb = min(nbits, bits.shape[1], 64)
    key = np.zeros(bits.shape[0], dtype=np.uint64)
    for p in range(nb):
        key |= bits[:, p].astype(np.uint64) << np.uint64(63 - p)
    return key


def root_subtree(words: np.ndarray, c: int) -> np.ndarray:
    """Integer formed by the first bit of each segment (segment 0 most significant)."""
    words = np.asarray(words, dtype=np.uint8)
    n, w = words.shape
    out = np.zeros(n, dtype=np.int64)
    for j in range(w):
        out = (out << 1) | ((words[:, j] >> (c - 1)) & 1).astype(np.int64)
    return out


def sorted_order(words: np.ndarray, c: int, key_bits: int = 64) -> np.ndarray:
    """Series ids ordered by (interleaved-key prefix of key_bits bits, id)."""
    key = key_prefix(words, c, key_bits)
    if key_bits < 64:
        key = key & ~np.uint64((1 << (64 - key_bits)) - 1)
    ids = np.arange(len(key), dtype=np.int64)
    return np.lexsort((ids, key))


def leaf_envelopes(words_sorted: np.ndarray, leaf_size: int):
    """Per-leaf, per-segment min and max symbol; leaf i = sorted rows [i*L, (i+1)*L)."""
    ws = np.asarray(words_sorted, dtype=np.uint8)
    n, w = ws.shape
    nl = (n + leaf_size - 1) // leaf_size
    lo = np.empty((nl, w), np.uint8)
    hi = np.empty((nl, w), np.uint8)
    for i in range(nl):
        blk = ws[i * leaf_size:(i + 1) * leaf_size]
        lo[i] = blk.min(axis=0)
        hi[i] = blk.max(axis=0)
    return lo, hi


def _region_edges(beta: np.ndarray):
    beta = np.asarray(beta, dtype=np.float64)
    lower = np.concatenate([[-np.inf], beta])   # lower[s] = beta_s
    upper = np.concatenate([beta, [np.inf]])    # upper[s] = beta_{s+1}
    return lower, upper


def mindist_sq(paa_q: np.ndarray, words: np.ndarray, beta: np.ndarray, m: int) -> np.ndarray:
    """Squared iSAX MINDIST of one query PAA against every word, FP64.

    LB^2 = m * sum_j dist(p_j, region of s_j)^2, where the distance of a point
    to the half-open region [beta_s, beta_{s+1}) is max(0, beta_s - p, p - beta_{s+1}).
    """
    lower, upper = _region_edges(beta)
    words = np.asarray(words, dtype=np.int64)
    p = np.asarray(paa_q, dtype=np.float64)[None, :]
    d = np.maximum(0.0, np.maximum(lower[words] - p, p - upper[words]))
    return m * (d * d).sum(axis=1)


def envelope_mindist_sq(paa_q, lo, hi, beta, m) -> np.ndarray:
    """Squared MINDIST of a query PAA to leaf envelopes [beta_lo, beta_{hi+1}) per segment."""
    lower, upper = _region_edges(beta)
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    p = np.asarray(paa_q, dtype=np.float64)[None, :]
    d = np.maximum(0.0, np.maximum(lower[lo] - p, p - upper[hi]))
    return m * (d * d).sum(axis=1)
