"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Inputs are seeded random walks (workload.py) generated on the device and
copied to the host for the oracle.  Bars: words, layout and ids bit-exact;
distances within 1e-4 relative of the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import workload
from oracle import isax_ref as ir
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu

RTOL = 1e-4


@pytest.fixture(scope="module")
def isax():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    return isax


def _cpu(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def coll(isax):
    # several leaf tiles (256 leaves x 256 series) and a ragged tail
    X = workload.random_walks(100_003, 256, seed=20090161, device="cuda")
    workload.planted_duplicates(X, [(99_999, 17), (50_000, 17), (1234, 777)])
    Q_noisy, src, sig = workload.noisy_queries(X, 9, seed=20091161)
    Q_fresh = workload.fresh_queries(4, 256, seed=20091161, device="cuda")
    Q = torch.cat([Q_noisy, Q_fresh, X[17:18].clone(), X[777:778].clone()]).contiguous()
    Xh, Qh = _cpu(X), _cpu(Q)
    ids10, d2_10 = kr.knn_exact_c(Xh, Qh, 10)
    return {"X": X, "Q": Q, "Xh": Xh, "Qh": Qh, "ids10": ids10, "d2_10": d2_10}


def _check_answer(ids, dists, ref_ids, ref_d2, k):
    ids, dists = _cpu(ids), _cpu(dists)
    assert np.array_equal(ids, ref_ids[:, :k]), (ids, ref_ids[:, :k])
    ref = np.sqrt(ref_d2[:, :k])
    err = np.abs(dists.astype(np.float64) - ref) / np.maximum(ref, 1e-30)
    err[ref == 0] = np.abs(dists[ref == 0])
    assert err.max() <= RTOL, err.max()


# ----------------------------------------------------------------------------- a1 summarise
@pytest.mark.parametrize("n,length,w,c", [(50_001, 256, 16, 8), (40_000, 128, 16, 8), (30_011, 256, 8, 4),
                                          (20_000, 64, 16, 3), (10_007, 48, 16, 8), (5_000, 256, 2, 8),
                                          (3_000, 96, 32, 6)])
def test_summarize_words_bit_exact(isax, n, length, w, c):
    X = workload.random_walks(n, length, seed=n + length, device="cuda")
    words, mx = isax.summarize(X, w, c)
    Xh = _cpu(X)
    assert np.array_equal(_cpu(words), ir.isax_words(Xh, w, c))
    assert mx == np.abs(Xh).max()


def test_summarize_symbols_agree_with_fp64_paa_away_from_edges(isax):
    X = workload.random_walks(20_000, 256, seed=5, device="cuda")
    words, mx = isax.summarize(X, 16, 8)
    Xh = _cpu(X)
    p64 = ir.paa64(Xh, 16)
    s64 = ir.symbols(p64, ir.breakpoints(8))
    diff = _cpu(words).astype(int) - s64.astype(int)
    beta = ir.breakpoints(8)
    near = np.min(np.abs(p64[..., None] - beta), axis=-1) <= 16 * 2.0 ** -23 * mx
    assert np.all(np.abs(diff) <= 1) and np.all(near[diff != 0])


# ----------------------------------------------------------------------------- a2 layout
@pytest.mark.parametrize("leaf,key_bits", [(256, 64), (64, 16), (1000, 40)])
def test_layout_matches_oracle(isax, leaf, key_bits):
    X = workload.random_walks(70_001, 128, seed=11, device="cuda")
    idx = isax.Index(X, 16, 8, leaf_size=leaf, key_bits=key_bits)
    ids, words, lo, hi = (_cpu(t) for t in idx.export())
    Xh = _cpu(X)
    wref = ir.isax_words(Xh, 16, 8)
    order = ir.sorted_order(wref, 8, key_bits)
    assert np.array_equal(ids, order)
    assert np.array_equal(words, wref[order])
    elo, ehi = ir.leaf_envelopes(wref[order], leaf)
    assert np.array_equal(lo, elo) and np.array_equal(hi, ehi)
    info = idx.info()
    assert info["n_leaves"] == (70_001 + leaf - 1) // leaf and info["max_abs"] == np.abs(Xh).max()


# ----------------------------------------------------------------------------- a3/a6 lower bounds
def test_lower_bounds_below_distance_and_near_mindist(isax, coll):
    X = coll["X"][:20_000].contiguous()
    idx = isax.Index(X, 16, 8)
    Q = coll["Q"]
    lb = _cpu(idx.lower_bounds(Q)).astype(np.float64)
    Xh = coll["Xh"][:20_000]
    words = ir.isax_words(Xh, 16, 8)
    beta = ir.breakpoints_f32(8).astype(np.float64)
    for j in range(Q.shape[0]):
        d2 = kr.sq_dists(Xh, coll["Qh"][j])
        assert np.all(lb[j] <= d2)
        ref = ir.mindist_sq(ir.paa64(coll["Qh"][j:j + 1], 16)[0], words, beta, 16)
        # the GPU widens every region by delta (~1e-5) and uses FP32 PAA
        assert np.all(np.abs(np.sqrt(lb[j]) - np.sqrt(ref)) <= 1e-3)


# ----------------------------------------------------------------------------- a4-a8 query
@pytest.mark.parametrize("mode", ["index", "scan"])
@pytest.mark.parametrize("k", [1, 10])
def test_query_parity(isax, coll, mode, k):
    idx = isax.Index(coll["X"], 16, 8)
    ids, d = idx.query(coll["Q"], k=k, mode=mode)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], k)


def test_duplicates_and_self_queries(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    ids, d = idx.query(coll["Q"][-2:].contiguous(), k=4)
    ids, d = _cpu(ids), _cpu(d)
    assert list(ids[0][:3]) == [17, 50_000, 99_999] and np.all(d[0][:3] == 0)
    assert list(ids[1][:2]) == [777, 1234] and np.all(d[1][:2] == 0)


@pytest.mark.parametrize("opts", [dict(leaf_size=16), dict(leaf_size=1024), dict(key_bits=16),
                                  dict(leaf_size=100, key_bits=24)])
def test_metamorphic_layouts(isax, coll, opts):
    idx = isax.Index(coll["X"], 16, 8, **opts)
    ids, d = idx.query(coll["Q"], k=10)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], 10)


@pytest.mark.parametrize("w,c", [(8, 8), (16, 4), (32, 2), (64, 8)])
def test_metamorphic_summaries(isax, coll, w, c):
    idx = isax.Index(coll["X"], w, c)
    ids, d = idx.query(coll["Q"], k=3)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], 3)


@pytest.mark.parametrize("flags", [1, 2, 3, 4, 7])
def test_sharing_and_abandon_switches(isax, coll, flags):
    idx = isax.Index(coll["X"], 16, 8)
    ids, d = idx.query(coll["Q"], k=10, flags=flags)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], 10)


def test_batches_and_order(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    perm = torch.randperm(coll["Q"].shape[0], generator=torch.Generator().manual_seed(3))
    ids, d = idx.query(coll["Q"][perm.cuda()].contiguous(), k=10, batch=4)
    inv = torch.argsort(perm)
    _check_answer(ids[inv.cuda()], d[inv.cuda()], coll["ids10"], coll["d2_10"], 10)


def test_k_prefix_and_per_query_k(isax, coll):
    idx = isax.Index(coll["X"], 16, 8)
    kq = torch.tensor([1 + (i % 10) for i in range(coll["Q"].shape[0])], dtype=torch.int32)
    ids, d = idx.query(coll["Q"], k=10, k_per_query=kq)
    ids, d = _cpu(ids), _cpu(d)
    for i, kk in enumerate(kq.tolist()):
        assert np.array_equal(ids[i, :kk], coll["ids10"][i, :kk])
        assert np.all(ids[i, kk:] == -1) and np.all(np.isinf(d[i, kk:]))


@pytest.mark.parametrize("mode", ["index", "scan"])
def test_candidate_overflow_fallback(isax, coll, mode):
    idx = isax.Index(coll["X"], 16, 8)
    ids, d = idx.query(coll["Q"], k=10, mode=mode, candidate_capacity=10)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], 10)


def test_small_collections_and_k_equals_n(isax):
    X = workload.random_walks(37, 64, seed=3, device="cuda")
    Q = workload.fresh_queries(5, 64, seed=4, device="cuda")
    ref_ids, ref_d2 = kr.knn_exact(_cpu(X), _cpu(Q), 37)
    for mode in ("index", "scan"):
        idx = isax.Index(X, 16, 8, leaf_size=16)
        ids, d = idx.query(Q, k=37, mode=mode)
        _check_answer(ids, d, ref_ids, ref_d2, 37)


def test_ragged_length_not_multiple_of_four(isax):
    X = workload.random_walks(5_003, 54, seed=7, device="cuda")
    Q = workload.fresh_queries(6, 54, seed=8, device="cuda")
    ref_ids, ref_d2 = kr.knn_exact(_cpu(X), _cpu(Q), 5)
    idx = isax.Index(X, 6, 8)
    for mode in ("index", "scan"):
        ids, d = idx.query(Q, k=5, mode=mode)
        _check_answer(ids, d, ref_ids, ref_d2, 5)


def test_errors_leave_outputs_untouched(isax, coll):
    X = coll["X"][:1000].clone()
    idx = isax.Index(X, 16, 8)
    Q = coll["Q"][:3].clone()
    Q[1, 5] = float("nan")
    ids = torch.full((3, 2), 7, dtype=torch.int64, device="cuda")
    d = torch.full((3, 2), 7.0, device="cuda")
    rc = isax.lib().isax_query(idx.handle, Q.data_ptr(), 3, 2, ids.data_ptr(), d.data_ptr())
    assert rc == isax.ISAX_EINVAL and "non-finite" in isax.last_error()
    assert torch.all(ids == 7) and torch.all(d == 7.0)
    X[10, 3] = float("inf")
    with pytest.raises(isax.IsaxError):
        isax.Index(X, 16, 8)
    with pytest.raises(isax.IsaxError):
        idx.query(coll["Q"][:3].contiguous(), k=1001)
    out = idx.query(coll["Q"][:0].contiguous(), k=1)
    assert out[0].shape == (0, 1)
    # pageable host memory is rejected before any device work
    host = np.zeros((100, 256), np.float32)
    assert not isax.lib().isax_build(host.ctypes.data, 100, 256, 16, 8)
    assert "not device memory" in isax.last_error()


def test_sorted_rows_copy(isax, coll):
    """With the FP32 rows also kept in leaf order, refinement reads them there; same answers."""
    plain = isax.Index(coll["X"], 16, 8, precision=1)
    idx = isax.Index(coll["X"], 16, 8, precision=5)
    inf, inf0 = idx.info(), plain.info()
    assert inf["has_sorted_rows"] == 1 and inf0["has_sorted_rows"] == 0
    assert inf["device_bytes"] - inf0["device_bytes"] >= coll["X"].numel() * 4
    for mode in ("index", "scan", "bf16"):
        ids, d = idx.query(coll["Q"], k=10, mode=mode)
        _check_answer(ids, d, coll["ids10"], coll["d2_10"], 10)
    ids, d = idx.query(coll["Q"], k=10, candidate_capacity=10)
    _check_answer(ids, d, coll["ids10"], coll["d2_10"], 10)
