"""Brute-force exact k-NN under Euclidean distance in FP64 (CPU oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The method of the paper prunes only series whose lower bound exceeds the
best-so-far distance and refines the rest with real distances (Sec. III,
ParIS/ParIS+ and MESSI query answering), so it reaches the plain definition
of the nearest neighbour (Sec. II, Similarity Search).  That definition is
what this module writes out:

  D_i = sum_{t=0}^{len-1} (q_t - x_{i,t})^2   in FP64, t in index order,
  answer = first k of the collection ordered by (D_i, i), distance sqrt(D_i).

Ties are broken by the lower series id.  `knn_exact` (numpy) and the C twin
`knn_ref.c` (driven by `knn_exact_c`) do the same arithmetic in the same order
and agree bit for bit; the C twin streams chunks and uses all host threads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libknn_ref.so")


def sq_dists(X: np.ndarray, q: np.ndarray) -> np.ndarray:
    """D_i for one query against all rows of X, FP64, accumulated over t in order."""
    X = np.asarray(X)
    q64 = np.asarray(q, dtype=np.float64)
    D = np.zeros(X.shape[0], dtype=np.float64)
    for t in range(X.shape[1]):
        d = q64[t] - X[:, t].astype(np.float64)
        D += d * d
    return D


def knn_exact(X: np.ndarray, Q: np.ndarray, k: int):
    """Exact k-NN: (ids int64 [m, k], squared distances float64 [m, k])."""
    X = np.asarray(X, dtype=np.float32)
    Q = np.asarray(Q, dtype=np.float32).reshape(-1, X.shape[1])
    n = X.shape[0]
    if not 1 <= k <= n:
        raise ValueError("k must be in 1..n")
    Xt = np.ascontiguousarray(X.T)          # column t of X is row t of Xt
    ids = np.empty((Q.shape[0], k), np.int64)
    d2 = np.empty((Q.shape[0], k), np.float64)
    all_ids = np.arange(n, dtype=np.int64)
    for j, q in enumerate(Q):
        q64 = q.astype(np.float64)
        D = np.zeros(n, dtype=np.float64)
        for t in range(Xt.shape[0]):
            d = q64[t] - Xt[t].astype(np.float64)
            D += d * d
        order = np.lexsort((all_ids, D))[:k]
        ids[j] = order
        d2[j] = D[order]
    return ids, d2


# ---------------------------------------------------------------- C twin
def build_c(force: bool = False) -> str:
    """Compile knn_ref.c into libknn_ref.so next to it (gcc, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "knn_ref.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", _SO, src, "-lm"])
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_c()
        lib = ctypes.CDLL(_SO)
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_knn_merge.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                         f32p, ctypes.c_int32, ctypes.c_int32, f64p, i64p]
        lib.oracle_knn_init.argtypes = [f64p, i64p, ctypes.c_int64]
        lib.oracle_sq_dists.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f32p, f64p]
        lib.oracle_dtw_sq.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f32p, ctypes.c_int32, f64p]
        lib.oracle_dtw_knn_merge.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                             f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, f64p, i64p]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class KnnState:
    """Running per-query top-k lists for streaming a collection through in chunks.

    window=None: Euclidean distance; window=r: DTW with band half-width r (dtw_ref).
    """

    def __init__(self, Q: np.ndarray, k: int, window: int | None = None):
        self.Q = np.ascontiguousarray(Q, dtype=np.float32)
        self.k = int(k)
        self.window = window
        m = self.Q.shape[0]
        self.d2 = np.empty((m, k), np.float64)
        self.ids = np.empty((m, k), np.int64)
        _load().oracle_knn_init(_ptr(self.d2, ctypes.c_double), _ptr(self.ids, ctypes.c_int64), m * k)

    def merge(self, X_chunk: np.ndarray, id_offset: int) -> None:
        X = np.ascontiguousarray(X_chunk, dtype=np.float32)
        if X.shape[1] != self.Q.shape[1]:
            raise ValueError("length mismatch")
        if self.window is None:
            _load().oracle_knn_merge(_ptr(X, ctypes.c_float), X.shape[0], X.shape[1], int(id_offset),
                                     _ptr(self.Q, ctypes.c_float), self.Q.shape[0], self.k,
                                     _ptr(self.d2, ctypes.c_double), _ptr(self.ids, ctypes.c_int64))
        else:
            _load().oracle_dtw_knn_merge(_ptr(X, ctypes.c_float), X.shape[0], X.shape[1], int(id_offset),
                                         _ptr(self.Q, ctypes.c_float), self.Q.shape[0], self.k, int(self.window),
                                         _ptr(self.d2, ctypes.c_double), _ptr(self.ids, ctypes.c_int64))


def knn_exact_c(X: np.ndarray, Q: np.ndarray, k: int):
    """Same result as knn_exact, computed by the C twin on all host threads."""
    st = KnnState(np.asarray(Q, np.float32).reshape(-1, np.asarray(X).shape[1]), k)
    st.merge(X, 0)
    return st.ids.copy(), st.d2.copy()


def sq_dists_c(X: np.ndarray, q: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    out = np.empty(X.shape[0], np.float64)
    _load().oracle_sq_dists(_ptr(X, ctypes.c_float), X.shape[0], X.shape[1],
                            _ptr(q, ctypes.c_float), _ptr(out, ctypes.c_double))
    return out


def knn_dtw_c(X: np.ndarray, Q: np.ndarray, k: int, window: int):
    """Same result as dtw_ref.knn_dtw, computed by the C twin on all host threads."""
    st = KnnState(np.asarray(Q, np.float32).reshape(-1, np.asarray(X).shape[1]), k, window)
    st.merge(X, 0)
    return st.ids.copy(), st.d2.copy()


def dtw_sq_c(X: np.ndarray, q: np.ndarray, window: int) -> np.ndarray:
    """Same values as dtw_ref.dtw_sq, by the C twin."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.float32)
    out = np.empty(X.shape[0], np.float64)
    _load().oracle_dtw_sq(_ptr(X, ctypes.c_float), X.shape[0], X.shape[1], _ptr(q, ctypes.c_float),
                          int(window), _ptr(out, ctypes.c_double))
    return out
