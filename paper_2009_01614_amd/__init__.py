"""Exact k-NN Euclidean search with an iSAX index on AMD Instinct MI355X.

Thin ctypes binding over the C ABI in include/isax.h (libisax.so, built from
csrc/ by build.py).  This module only marshals arguments: every step of index
build and query answering runs in the library's HIP kernels.  PyTorch tensors
provide device memory and the current stream.  If the library is missing the
import fails; there is no fallback.

    idx = Index(data)                         # data: cuda FP32 [n, len]
    ids, dists = idx.query(queries, k=10)     # exact, ascending, ties by lower id
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisax.so")

ISAX_OK, ISAX_EINVAL, ISAX_ENOMEM, ISAX_EDEVICE, ISAX_EOVERFLOW = 0, -1, -2, -3, -4
MODE_INDEX, MODE_SCAN, MODE_BF16, MODE_FP8, MODE_HYBRID = 0, 1, 2, 3, 4
MODES = {"index": MODE_INDEX, "scan": MODE_SCAN, "bf16": MODE_BF16, "fp8": MODE_FP8, "hybrid": MODE_HYBRID}
METRIC_ED, METRIC_DTW = 0, 1
METRICS = {"ed": METRIC_ED, "dtw": METRIC_DTW}
MAX_WINDOW = 31
QF_NO_SHARING, QF_NO_EARLY_ABANDON, QF_NO_BEST_FIRST, QF_NO_SHORTCUT, QF_FILTER_CHEAP, QF_FILTER_DEAR = 1, 2, 4, 8, 16, 32
QF_FULL_ROWS, QF_NO_PRECHECK = 64, 128
# isax_build_options.precision bits
PREC_BF16, PREC_FP8, PREC_SORTED_ROWS, PREC_SPECTRAL = 1, 2, 4, 8
SERVE_BATCHES = 1
EDGES = {"normal": 0, "empirical": 1}
MAX_K = 1024


class IsaxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"isax error {code}: {msg}")
        self.code = code


class BuildOptions(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("key_bits", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("edges", ctypes.c_int32), ("stream", ctypes.c_void_p), ("spectral_dim", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class QueryStats(ctypes.Structure):
    _fields_ = [("leaves_scanned", ctypes.c_int64), ("leaves_kept", ctypes.c_int64),
                ("series_bounded", ctypes.c_int64), ("series_refined", ctypes.c_int64),
                ("refine_bytes", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("tau_initial", ctypes.c_float), ("tau_final", ctypes.c_float),
                ("dtw_series", ctypes.c_int64), ("dtw_cells", ctypes.c_int64),
                ("leaves_initial", ctypes.c_int64), ("path", ctypes.c_int32),
                ("candidate_capacity", ctypes.c_int32)]


class QueryOptions(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("candidate_capacity", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("k_per_query", ctypes.c_void_p), ("stream", ctypes.c_void_p),
                ("stats", ctypes.POINTER(QueryStats)), ("metric", ctypes.c_int32), ("window", ctypes.c_int32),
                ("hybrid_leaves", ctypes.c_int64)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("len", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("card_bits", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("key_bits", ctypes.c_int32),
                ("has_bf16", ctypes.c_int32), ("has_fp8", ctypes.c_int32), ("n_leaves", ctypes.c_int64),
                ("max_abs", ctypes.c_float), ("delta", ctypes.c_float), ("device_bytes", ctypes.c_int64),
                ("has_sorted_rows", ctypes.c_int32), ("edges", ctypes.c_int32), ("spectral_dim", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("algorithmic_bytes", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("streams", ctypes.c_int32), ("memory_budget", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("flags", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("k", ctypes.c_int32),
                ("collection", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double), ("ids", ctypes.c_int64 * MAX_K),
                ("dists", ctypes.c_float * MAX_K), ("message", ctypes.c_char * 120)]


# name -> (restype, argtypes); mirrors include/isax.h
_VP, _I32, _I64, _F32P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "isax_last_error": (ctypes.c_char_p, []),
    "isax_build": (_VP, [_VP, _I64, _I32, _I32, _I32]),
    "isax_build_ex": (_VP, [_VP, _I64, _I32, _I32, _I32, ctypes.POINTER(BuildOptions)]),
    "isax_free": (None, [_VP]),
    "isax_query": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP]),
    "isax_query_ex": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP, ctypes.POINTER(QueryOptions)]),
    "isax_query_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP, ctypes.POINTER(QueryOptions)]),
    "isax_breakpoints": (ctypes.c_int, [_I32, _F32P]),
    "isax_summarize": (ctypes.c_int, [_VP, _I64, _I32, _I32, _I32, _VP, _F32P, _VP]),
    "isax_index_get_info": (ctypes.c_int, [_VP, ctypes.POINTER(IndexInfo)]),
    "isax_index_breakpoints": (ctypes.c_int, [_VP, _F32P]),
    "isax_host_alloc": (ctypes.c_void_p, [ctypes.c_int64]),
    "isax_host_free": (None, [_VP]),
    "isax_index_export": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "isax_lower_bounds": (ctypes.c_int, [_VP, _VP, _I64, _VP]),
    "isax_filter_scores": (ctypes.c_int, [_VP, _VP, _I64, _I32, _VP, _VP]),
    "isax_profile_enable": (ctypes.c_int, [_I32]),
    "isax_profile_read": (ctypes.c_int, [ctypes.POINTER(ProfileEntry), _I32, ctypes.POINTER(ctypes.c_int32)]),
    "isax_profile_reset": (ctypes.c_int, []),
    "isax_server_create": (_VP, [ctypes.POINTER(_VP), _I32, ctypes.POINTER(ServerOptions)]),
    "isax_server_submit": (ctypes.c_int, [_VP, _I32, _F32P, _I32, ctypes.c_uint64]),
    "isax_server_poll": (ctypes.c_int, [_VP, ctypes.POINTER(Result), _I32, _I32]),
    "isax_server_pending": (_I64, [_VP]),
    "isax_server_destroy": (None, [_VP]),
    "isax_clock": (ctypes.c_double, []),
    "isax_debug_fail_allocation": (ctypes.c_int, [_I64]),
}

_lib = None


def lib():
    """The loaded libisax.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_01614_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().isax_last_error().decode()


def _check(rc: int):
    if rc != ISAX_OK:
        raise IsaxError(rc, last_error())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t: torch.Tensor, name: str, allow_pinned: bool = False) -> torch.Tensor:
    where = t.is_cuda or (allow_pinned and t.is_pinned())
    if not (where and t.dtype == torch.float32 and t.dim() == 2 and t.is_contiguous()):
        kind = "CUDA or pinned host" if allow_pinned else "CUDA"
        raise ValueError(f"{name} must be a contiguous 2-D float32 {kind} tensor")
    return t


class HostRows:
    """Page-locked host memory from isax_host_alloc holding an FP32 [n, len] collection.

    `tensor` is a CPU tensor over that memory (for filling it and for Index).  The tensor
    holds this object, so the memory lives as long as the tensor or anything keeping it (an
    Index keeps its data tensor); close() releases it at once, and must not be called
    while an index over the rows is still in use."""

    def __init__(self, n: int, length: int):
        import numpy as np
        nbytes = int(n) * int(length) * 4
        p = lib().isax_host_alloc(nbytes)
        if not p:
            raise IsaxError(ISAX_ENOMEM, last_error())
        self._p = p
        arr = np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_float)), shape=(int(n), int(length)))
        self.tensor = torch.from_numpy(arr)
        self.tensor._isax_host_rows = self  # the owner lives as long as the tensor

    def close(self):
        if getattr(self, "_p", None):
            self.tensor = None
            lib().isax_host_free(ctypes.c_void_p(self._p))
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- host-side helpers
def breakpoints(card_bits: int):
    """The 2^c - 1 FP32 region edges the library uses."""
    import numpy as np
    out = np.empty((1 << card_bits) - 1, np.float32)
    _check(lib().isax_breakpoints(card_bits, out.ctypes.data_as(_F32P)))
    return out


def summarize(data: torch.Tensor, segments: int = 16, card_bits: int = 8, stream=None):
    """(words uint8 [n, segments] on the device, max |x|) without building an index."""
    _dev_f32(data, "data")
    n, length = data.shape
    words = torch.empty((n, segments), dtype=torch.uint8, device=data.device)
    mx = ctypes.c_float(0)
    _check(lib().isax_summarize(data.data_ptr(), n, length, segments, card_bits, words.data_ptr(),
                                ctypes.byref(mx), _stream(stream)))
    return words, mx.value


def profile_enable(on: bool = True):
    _check(lib().isax_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().isax_profile_reset())


def profile_read() -> dict:
    """{kernel name: {'launches', 'total_ms', 'algorithmic_bytes'}} accumulated since the last reset."""
    buf = (ProfileEntry * 128)()
    n = ctypes.c_int32(0)
    _check(lib().isax_profile_read(buf, 128, ctypes.byref(n)))
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "algorithmic_bytes": buf[i].algorithmic_bytes} for i in range(min(n.value, 128))}


# ----------------------------------------------------------------------------- index
class Index:
    """An iSAX index over a resident FP32 collection (the tensor is borrowed, keep it alive).

    The collection may sit in device memory or in pinned host memory (read over
    the bus; the summaries, the layout and any reduced-precision copy are in HBM).
    """

    def __init__(self, data: torch.Tensor, segments: int = 16, card_bits: int = 8, leaf_size: int = 0,
                 key_bits: int = 0, precision: int = 0, stream=None, edges="normal", spectral_dim: int = 0):
        """edges: "normal" (standard-normal quantiles) or "empirical" (the collection's own).
        precision: bits PREC_*; spectral_dim: D of the spectral copy (PREC_SPECTRAL), 0 = the default."""
        _dev_f32(data, "data", allow_pinned=True)
        self.data = data
        self.n, self.len = data.shape
        self.card_bits = card_bits
        opt = BuildOptions(leaf_size, key_bits, precision, EDGES[edges] if isinstance(edges, str) else int(edges),
                           _stream(stream), spectral_dim, 0)
        h = lib().isax_build_ex(data.data_ptr(), self.n, self.len, segments, card_bits, ctypes.byref(opt))
        if not h:
            raise IsaxError(ISAX_EINVAL, last_error())
        self._h = ctypes.c_void_p(h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().isax_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def breakpoints(self):
        """The index's 2^c - 1 region edges (numpy FP32)."""
        import numpy as np
        out = np.zeros((1 << self.card_bits) - 1, np.float32)
        _check(lib().isax_index_breakpoints(self._h, out.ctypes.data_as(_F32P)))
        return out

    def info(self) -> dict:
        inf = IndexInfo()
        _check(lib().isax_index_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in IndexInfo._fields_}

    def export(self):
        """(ids_sorted int32 [n], words_sorted uint8 [n, w], env_lo, env_hi uint8 [n_leaves, w]) on the device."""
        inf = self.info()
        dev = self.data.device if self.data.is_cuda else torch.device("cuda", torch.cuda.current_device())
        ids = torch.empty(self.n, dtype=torch.int32, device=dev)
        words = torch.empty((self.n, inf["segments"]), dtype=torch.uint8, device=dev)
        lo = torch.empty((inf["n_leaves"], inf["segments"]), dtype=torch.uint8, device=dev)
        hi = torch.empty_like(lo)
        _check(lib().isax_index_export(self._h, ids.data_ptr(), words.data_ptr(), lo.data_ptr(), hi.data_ptr()))
        return ids, words, lo, hi

    def query(self, queries: torch.Tensor, k: int = 1, mode="index", k_per_query: torch.Tensor | None = None,
              candidate_capacity: int = 0, flags: int = 0, batch: int = 0, stream=None, stats: bool = False,
              metric="ed", window: int = 0, hybrid_leaves: int = 0, noalloc: bool = False):
        """Exact k-NN: (ids int64 [m, k], dists float32 [m, k]); with stats=True also a list of dicts.

        noalloc=True calls isax_query_noalloc (no device allocation inside the call; scratch from the
        library's fixed per-device array).

        metric "ed" (Euclidean) or "dtw" (banded DTW of half-width `window`, modes "index" and "scan").
        mode "hybrid" answers each query with the iSAX path or the BF16 filter, by the leaves the iSAX
        path would still bound after its first round: above `hybrid_leaves`, or (0) by the library's
        cost model.
        """
        _dev_f32(queries, "queries")
        m = queries.shape[0]
        if queries.shape[1] != self.len:
            raise ValueError("query length differs from the collection's")
        ids = torch.empty((m, k), dtype=torch.int64, device=queries.device)
        dists = torch.empty((m, k), dtype=torch.float32, device=queries.device)
        st = (QueryStats * max(m, 1))() if stats else None
        kp = None
        if k_per_query is not None:
            k_per_query = k_per_query.to(device=queries.device, dtype=torch.int32).contiguous()
            kp = k_per_query.data_ptr()
        opt = QueryOptions(MODES[mode] if isinstance(mode, str) else int(mode), candidate_capacity, flags, batch,
                           kp, _stream(stream), st, METRICS[metric] if isinstance(metric, str) else int(metric),
                           window, hybrid_leaves)
        fn = lib().isax_query_noalloc if noalloc else lib().isax_query_ex
        _check(fn(self._h, queries.data_ptr(), m, k, ids.data_ptr(), dists.data_ptr(), ctypes.byref(opt)))
        if stats:
            return ids, dists, [{f: getattr(st[i], f) for f, _ in QueryStats._fields_} for i in range(m)]
        return ids, dists

    def lower_bounds(self, queries: torch.Tensor) -> torch.Tensor:
        """Squared iSAX lower bounds [m, n] (column = series id) used for pruning."""
        _dev_f32(queries, "queries")
        out = torch.empty((queries.shape[0], self.n), dtype=torch.float32, device=queries.device)
        _check(lib().isax_lower_bounds(self._h, queries.data_ptr(), queries.shape[0], out.data_ptr()))
        return out

    def filter_scores(self, queries: torch.Tensor, mode="bf16"):
        """(approx, margin) [m, n] of the reduced-precision filter, column = series id."""
        _dev_f32(queries, "queries")
        m = queries.shape[0]
        approx = torch.empty((m, self.n), dtype=torch.float32, device=queries.device)
        margin = torch.empty_like(approx)
        _check(lib().isax_filter_scores(self._h, queries.data_ptr(), m, MODES[mode] if isinstance(mode, str) else mode,
                                        approx.data_ptr(), margin.data_ptr()))
        return approx, margin


# ----------------------------------------------------------------------------- serving
class Server:
    """Continuous-batching request loop over resident indexes (see isax_server_* in include/isax.h)."""

    def __init__(self, indexes, max_batch: int = 0, streams: int = 0, memory_budget: int = 0, mode="index",
                 batches: bool = False, chunks: int = 0):
        """Step-level admission in the filter modes unless batches=True (see isax_server_* in isax.h)."""
        self.indexes = list(indexes)
        arr = (ctypes.c_void_p * len(self.indexes))(*[ix.handle.value for ix in self.indexes])
        opt = ServerOptions(max_batch, streams, memory_budget, MODES[mode] if isinstance(mode, str) else mode,
                            SERVE_BATCHES if batches else 0, chunks, 0)
        h = lib().isax_server_create(arr, len(self.indexes), ctypes.byref(opt))
        if not h:
            raise IsaxError(ISAX_EINVAL, last_error())
        self._h = ctypes.c_void_p(h)
        self._buf = (Result * 256)()

    def submit(self, collection: int, query, k: int, tag: int):
        import numpy as np
        q = np.ascontiguousarray(query, dtype=np.float32)
        _check(lib().isax_server_submit(self._h, collection, q.ctypes.data_as(_F32P), k, tag))

    def poll(self, timeout_ms: int = 0) -> list:
        n = lib().isax_server_poll(self._h, self._buf, len(self._buf), timeout_ms)
        if n < 0:
            raise IsaxError(n, last_error())
        out = []
        for i in range(n):
            r = self._buf[i]
            out.append({"tag": r.tag, "status": r.status, "k": r.k, "collection": r.collection,
                        "batch_size": r.batch_size, "t_submit": r.t_submit, "t_start": r.t_start,
                        "t_done": r.t_done, "ids": list(r.ids[:r.k]), "dists": list(r.dists[:r.k]),
                        "message": r.message.decode(errors="replace")})
        return out

    def pending(self) -> int:
        return int(lib().isax_server_pending(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().isax_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def clock() -> float:
    return lib().isax_clock()


def debug_fail_allocation(countdown: int):
    """Tests only: the countdown-th device allocation of the library from now on fails (0: off)."""
    _check(lib().isax_debug_fail_allocation(int(countdown)))
