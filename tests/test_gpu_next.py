"""Extensions beyond the in-HBM random-walk collections, same exactness bar.

* Embedding vectors (high-dimensional, not z-normalised): the index, the
  reduced-precision filter and the scan all return the oracle's answer, with
  the standard-normal region edges and with edges taken from the collection's
  own segment means (bit-exact against the oracle's, and so are the words).
* Raw data larger than device memory: the collection stays in pinned host
  memory (the library borrows the pointer and reads it over the bus); only the
  summaries, the leaf layout and the query state live in HBM.
"""
import numpy as np
import pytest
import torch

import workload
from oracle import isax_ref as ir
from oracle import knn_ref as kr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def isax():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_01614_amd as isax
    isax.lib()
    return isax


@pytest.mark.parametrize("dim", [128, 384])
def test_embedding_vectors(isax, dim):
    g = torch.Generator(device="cuda").manual_seed(dim)
    # clustered embeddings: 200 centres, anisotropic spread, not normalised
    centres = torch.randn(200, dim, device="cuda", generator=g) * 3.0
    lab = torch.randint(0, 200, (60_000,), device="cuda", generator=g)
    X = (centres[lab] + torch.randn(60_000, dim, device="cuda", generator=g) * 0.7).float().contiguous()
    Q = (centres[torch.randint(0, 200, (24,), device="cuda", generator=g)] +
         torch.randn(24, dim, device="cuda", generator=g) * 0.7).float().contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(X.cpu().numpy(), Q.cpu().numpy(), 10)
    idx = isax.Index(X, 16, 8, precision=3)
    for mode in ("index", "scan", "bf16", "fp8"):
        ids, d = idx.query(Q, k=10, mode=mode)
        assert np.array_equal(ids.cpu().numpy(), ref_ids), mode
        assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0), mode


def _embeddings(dim, n, m, seed, unit=False, spread=0.7):
    """Clustered vectors around 200 centres; unit=True scales every vector to norm 1."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((200, dim)) * (1.0 if unit else 3.0)
    X = centres[rng.integers(0, 200, n)] + spread * rng.standard_normal((n, dim))
    Q = centres[rng.integers(0, 200, m)] + spread * rng.standard_normal((m, dim))
    if unit:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return X.astype(np.float32), Q.astype(np.float32)


@pytest.mark.parametrize("dim,n,unit", [(128, 70_001, False), (384, 30_000, True)])
def test_empirical_edges_words_and_parity(isax, dim, n, unit):
    # w = dim / 8 segments; n = 70001 > 65536 / 16 exercises the evenly spaced sample
    w = dim // 8
    Xh, Qh = _embeddings(dim, n, 20, 1000 + dim, unit=unit, spread=0.5 if unit else 0.7)
    X, Q = torch.from_numpy(Xh).cuda(), torch.from_numpy(Qh).cuda()
    idx = isax.Index(X, w, 8, precision=3, edges="empirical")
    assert idx.info()["edges"] == isax.EDGES["empirical"]
    e = ir.empirical_breakpoints(Xh, w, 8)
    assert np.array_equal(idx.breakpoints(), e)
    ids_s, words_s, _, _ = (t.cpu().numpy() for t in idx.export())
    want = ir.isax_words(Xh, w, 8, e)
    assert np.array_equal(words_s, want[ids_s])
    # the edges spread the symbols evenly over the 256 regions
    h = np.bincount(want.ravel(), minlength=256) / want.size
    assert h.max() < 4.0 / 256
    # lower bounds stay below the distances and near the oracle's MINDIST with these edges
    lb = idx.lower_bounds(Q).cpu().numpy().astype(np.float64)
    for j in range(0, 20, 5):
        d2 = kr.sq_dists(Xh, Qh[j])
        assert np.all(lb[j] <= d2)
        ref = ir.mindist_sq(ir.paa64(Qh[j:j + 1], w)[0], want, e.astype(np.float64), 8)
        assert np.all(np.abs(np.sqrt(lb[j]) - np.sqrt(ref)) <= 1e-3 * max(1.0, float(np.abs(Xh).max())))
    ref_ids, ref_d2 = kr.knn_exact_c(Xh, Qh, 10)
    for mode in ("index", "scan", "bf16", "fp8", "hybrid"):
        ids, d = idx.query(Q, k=10, mode=mode)
        assert np.array_equal(ids.cpu().numpy(), ref_ids), mode
        assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0), mode


def test_empirical_edges_tighten_bounds_on_unit_vectors(isax):
    # unit-norm vectors: with the standard-normal edges one symbol holds 12 % of the
    # segments; the collection's own edges leave about 6 % fewer series with a lower
    # bound under the 10th-NN distance on this seed (oracle: 53023 against 56575 per query)
    Xh, Qh = _embeddings(128, 60_000, 8, 5, unit=True, spread=0.5)
    X, Q = torch.from_numpy(Xh).cuda(), torch.from_numpy(Qh).cuda()
    _, ref_d2 = kr.knn_exact_c(Xh, Qh, 10)
    alive = {}
    for edges in ("normal", "empirical"):
        lb = isax.Index(X, 16, 8, edges=edges).lower_bounds(Q).cpu().numpy().astype(np.float64)
        alive[edges] = int((lb < ref_d2[:, -1:]).sum())
    assert alive["empirical"] < 0.97 * alive["normal"]


def test_raw_data_in_pinned_host_memory(isax):
    Xd = workload.random_walks(200_003, 256, seed=61, device="cuda")
    Xh = torch.empty(Xd.shape, dtype=torch.float32, pin_memory=True)
    Xh.copy_(Xd.cpu())
    del Xd
    Qn, _, _ = workload.noisy_queries(Xh.cuda(), 12, seed=62)
    Q = Qn.contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(Xh.numpy(), Q.cpu().numpy(), 5)
    import ctypes
    # the index borrows the host pointer; build and queries read it from the device
    opt = isax.BuildOptions(0, 0, 0, 0, None)
    h = isax.lib().isax_build_ex(Xh.data_ptr(), Xh.shape[0], 256, 16, 8, ctypes.byref(opt))
    assert h, isax.last_error()
    try:
        for mode in (isax.MODE_INDEX, isax.MODE_SCAN):
            ids = torch.empty((12, 5), dtype=torch.int64, device="cuda")
            d = torch.empty((12, 5), dtype=torch.float32, device="cuda")
            qo = isax.QueryOptions(mode, 0, 0, 0, None, None, None)
            rc = isax.lib().isax_query_ex(ctypes.c_void_p(h), Q.data_ptr(), 12, 5, ids.data_ptr(), d.data_ptr(),
                                          ctypes.byref(qo))
            assert rc == 0, isax.last_error()
            assert np.array_equal(ids.cpu().numpy(), ref_ids)
            assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0)
    finally:
        isax.lib().isax_free(ctypes.c_void_p(h))


@pytest.mark.parametrize("k", [1, 10])
def test_host_rows_with_bf16_precheck(isax, k):
    # pinned host rows with the BF16 copy in HBM: the approximate answer and the iSAX
    # refinement bound each series with the copy first and read only the rows that can
    # matter; answers are the oracle's in every mode
    Xd = workload.random_walks(200_003, 256, seed=63, device="cuda")
    workload.planted_duplicates(Xd, [(150_000, 7)])
    Xh = torch.empty(Xd.shape, dtype=torch.float32, pin_memory=True)
    Xh.copy_(Xd.cpu())
    Qn, _, _ = workload.noisy_queries(Xd, 30, seed=64)
    Q = torch.cat([Qn, Xd[7:8].clone()]).contiguous()
    ref_ids, ref_d2 = kr.knn_exact_c(Xh.numpy(), Q.cpu().numpy(), k)
    dev = isax.Index(Xd, 16, 8, precision=isax.PREC_BF16)
    host = isax.Index(Xh, 16, 8, precision=isax.PREC_BF16)
    for mode in ("index", "bf16", "hybrid"):
        ids, d, st = host.query(Q, k=k, mode=mode, stats=True)
        assert np.array_equal(ids.cpu().numpy(), ref_ids), mode
        assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0), mode
        ids2, d2 = dev.query(Q, k=k, mode=mode)
        assert torch.equal(ids, ids2) and torch.equal(d, d2), mode
    # rows read over the bus: far fewer than the device path refines
    _, _, st_h = host.query(Q, k=k, mode="index", stats=True)
    _, _, st_d = dev.query(Q, k=k, mode="index", stats=True)
    read_h = sum(s["series_refined"] for s in st_h)
    read_d = sum(s["series_refined"] for s in st_d)
    assert read_h < 0.5 * read_d, (read_h, read_d)
    del Xd


@pytest.mark.parametrize("flags", [0, 1, 4])  # plain, no sharing, no best-first
def test_precheck_on_device_data(isax, flags):
    # the precheck is on by default with the full-row BF16 copy; ISAX_QF_NO_PRECHECK reads rows directly
    X = workload.random_walks(150_001, 256, seed=65, device="cuda")
    Qn, _, _ = workload.noisy_queries(X, 40, seed=66)
    Q = torch.cat([Qn, workload.fresh_queries(4, 256, seed=67, device="cuda")]).contiguous()
    idx = isax.Index(X, 16, 8, precision=isax.PREC_BF16)
    ref_ids, ref_d2 = kr.knn_exact_c(X.cpu().numpy(), Q.cpu().numpy(), 10)
    for k in (1, 10):
        a, da, sa = idx.query(Q, k=k, mode="index", flags=flags | isax.QF_NO_PRECHECK, stats=True)
        b, db, sb = idx.query(Q, k=k, mode="index", flags=flags, stats=True)
        assert np.array_equal(b.cpu().numpy(), ref_ids[:, :k])
        assert torch.equal(a, b) and torch.equal(da, db)
        assert sum(s["series_refined"] for s in sb) <= sum(s["series_refined"] for s in sa)


def test_host_alloc_rows(isax):
    # rows in page-locked memory from isax_host_alloc (filled from the device), the
    # index over them answers as the oracle; a size of zero is refused
    n, L = 120_007, 256
    rows = isax.HostRows(n, L)
    try:
        Xd = workload.random_walks(n, L, seed=68, device="cuda")
        rows.tensor.copy_(Xd.cpu())
        Qn, _, _ = workload.noisy_queries(Xd, 20, seed=69)
        Q = Qn.contiguous()
        del Xd
        ref_ids, ref_d2 = kr.knn_exact_c(rows.tensor.numpy(), Q.cpu().numpy(), 10)
        idx = isax.Index(rows.tensor, 16, 8, precision=isax.PREC_BF16)
        for mode in ("index", "bf16", "hybrid"):
            ids, d = idx.query(Q, k=10, mode=mode)
            assert np.array_equal(ids.cpu().numpy(), ref_ids), mode
            assert np.allclose(d.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0), mode
        idx.close()
    finally:
        rows.close()
    with pytest.raises(isax.IsaxError, match="bytes must be > 0"):
        isax.HostRows(0, 256)


def test_host_rows_live_as_long_as_their_tensor(isax):
    # an index keeps its data tensor, and the tensor keeps the page-locked block: dropping
    # the HostRows object itself must not release memory the index still reads
    import gc
    import weakref
    rows = isax.HostRows(30_011, 128)
    owner = weakref.ref(rows)
    t = rows.tensor
    del rows
    gc.collect()
    assert owner() is not None, "the page-locked block was released while its tensor lives"
    Xd = workload.random_walks(30_011, 128, seed=70, device="cuda")
    t.copy_(Xd.cpu())
    Q = workload.noisy_queries(Xd, 8, seed=71)[0].contiguous()
    idx = isax.Index(t, 16, 8)
    del t
    gc.collect()
    assert owner() is not None
    ref_ids, _ = kr.knn_exact_c(Xd.cpu().numpy(), Q.cpu().numpy(), 5)
    ids, _ = idx.query(Q, k=5, mode="index")
    assert np.array_equal(ids.cpu().numpy(), ref_ids)
    idx.close()
    del idx
    gc.collect()
    assert owner() is None, "the block outlived every user"


def test_precheck_choice_on_clustered_vectors(isax):
    # 384-dimensional clustered vectors, 16 segments: early abandoning stops most FP32
    # rows after their first step, so waves mostly skip the precheck; answers are the
    # oracle's and the same with the precheck switched off
    g = torch.Generator(device="cuda").manual_seed(384)
    centres = torch.randn(200, 384, device="cuda", generator=g) * 3.0
    lab = torch.randint(0, 200, (60_001,), device="cuda", generator=g)
    E = (centres[lab] + torch.randn(60_001, 384, device="cuda", generator=g) * 0.7).contiguous()
    Q = (centres[torch.randint(0, 200, (40,), device="cuda", generator=g)] +
         torch.randn(40, 384, device="cuda", generator=g) * 0.7).contiguous()
    idx = isax.Index(E, 16, 8, precision=isax.PREC_BF16)
    ref_ids, ref_d2 = kr.knn_exact_c(E.cpu().numpy(), Q.cpu().numpy(), 10)
    a, da = idx.query(Q, k=10, mode="index")
    b, db = idx.query(Q, k=10, mode="index", flags=isax.QF_NO_PRECHECK)
    assert np.array_equal(a.cpu().numpy(), ref_ids)
    assert np.allclose(da.cpu().numpy(), np.sqrt(ref_d2), rtol=1e-4, atol=0)
    assert torch.equal(a, b) and torch.equal(da, db)
