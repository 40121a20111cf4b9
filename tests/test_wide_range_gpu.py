"""Wide-range weights: scores many orders of magnitude below the query's largest product.

The doc-tiled kernels sum fp32 and bf16 products in fixed point with one scale per
query, so their error is absolute. A query whose k-th score is tiny beside its
largest product (query {A: 3, B: 1e-5, C: 1e-9} over docs holding B or C with
weights near 1e-5 or 1e-9, and k above the document frequency of A) must still meet
the fp32 rule (1e-5 relative) and the bf16 rule (ids and fp64 scores exact). The
selection detects those queries and sums their rows again in fp64; the diagnostics
say which queries took that pass. Every kernel is checked against the oracle.
"""
import numpy as np
import pytest

from helpers import csr
from parity_rules import check_batch

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


A, B, C = 0, 1, 2


def _collection(n_docs=270_000, vocab=64, seed=17):
    # 270K docs: 33 doc tiles of 8192 (17 of 16384), enough for fused candidate filtering
    rng = np.random.default_rng(seed)
    rows = [[] for _ in range(n_docs)]
    d = np.arange(n_docs)
    for x in d[d % 400 == 0]:  # 675 docs: weights in [0.5, 3]
        rows[x].append((A, float(rng.uniform(0.5, 3.0))))
    for x in d[d % 8 == 3]:  # 33,750 docs near 1e-5
        rows[x].append((B, float(1e-5 * rng.uniform(0.5, 2.0))))
    for x in d[d % 13 == 5]:  # 20,770 docs near 1e-9
        rows[x].append((C, float(1e-9 * rng.uniform(0.5, 2.0))))
    n_extra = rng.integers(0, 5, size=n_docs)
    for x in d:  # ordinary terms
        for t in rng.choice(np.arange(3, vocab), size=int(n_extra[x]), replace=False):
            rows[x].append((int(t), float(np.log1p(rng.lognormal(0.0, 0.8)))))
    return csr([sorted(r) for r in rows], vocab)


def _queries(vocab=64, seed=18):
    rng = np.random.default_rng(seed)
    rows, ks, wide = [], [], []
    # (terms, k, expected wide): k above df(A) = 675 puts the k-th score among the B-only
    # docs (~1e-10) or the C-only docs (~1e-18)
    special = [([(A, 3.0), (B, 1e-5), (C, 1e-9)], 1000, True),
               ([(A, 3.0), (B, 1e-5), (C, 1e-9)], 700, True),
               ([(A, 2.5), (B, 3e-5), (C, 1e-9)], 1024, True),
               ([(A, 3.0), (C, 1e-9)], 900, True),
               ([(A, 3.0), (B, 1e-5)], 300, False),  # k-th score among the A docs
               ([(A, 2.5), (B, 3e-5), (C, 1e-9), (7, 0.3)], 1000, False),  # among term 7's docs
               ([(B, 1e-5), (C, 1e-9)], 1000, None)]  # scale from B: C-only scores ~5e-9 of it
    for terms, k, wd in special:
        rows.append(terms)
        ks.append(k)
        wide.append(wd)
    while len(rows) < 40:  # ordinary queries (fused filtering runs on searches of 32+ queries)
        t = sorted(rng.choice(np.arange(3, vocab), size=int(rng.integers(1, 8)), replace=False).tolist())
        rows.append([(int(x), float(np.log1p(rng.lognormal(0.0, 0.8)))) for x in t])
        ks.append(int(rng.choice([10, 100, 1000])))
        wide.append(False)
    return csr(rows, vocab), np.array(ks, np.int32), wide


@pytest.fixture(scope="module")
def data():
    return _collection(), _queries()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("kernel", ["tiled", "shared", "group", "atomic", "docpar"])
@pytest.mark.parametrize("fused", [True, False])
def test_wide_range_weights_meet_the_rules(data, precision, kernel, fused):
    gs, torch = _gs()
    docs, (qs, ks, wide) = data
    if kernel in ("atomic", "docpar") and not fused:
        pytest.skip("fused filtering applies to the doc-tiled kernels only")
    idx = gs.Index.from_rows(docs, precision, keep_forward=(kernel == "docpar"),
                              keep_doc_ids=(kernel == "atomic"))
    b = idx.batch(qs, ks, k_max=1024)
    opts = gs.make_opts(kernel, fused_filter=fused)
    ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
    torch.cuda.synchronize()
    diag = b.diagnostics()
    assert diag[:, 3].max() == 0, "band overflow"
    check_batch(precision, docs, qs, ids.cpu().numpy(), sc.cpu().numpy(), ks, what="%s %s" % (precision, kernel))
    if kernel in ("tiled", "shared", "group"):
        # The fixed-point kernels sum the wide-range queries again in fp64. Without fused
        # filtering no other query takes that pass. With it, a query is checked against the
        # k-th score of the seed tiles (a lower bound; a fused query counts no other tile):
        # query 4 ({A, B}, k = 300) has fewer than 300 A docs there, so its bound falls among
        # the B-only docs and it may take the pass too (the check is conservative, the result
        # the same).
        for q, wd in enumerate(wide):
            if wd is True:
                assert diag[q, 4] == 2, "query %d was not summed in fp64" % q
            elif wd is False and not (fused and q == 4):
                assert diag[q, 4] != 2, "query %d was summed in fp64 without need" % q
    else:
        assert np.all(diag[:, 4] != 2), "fp32-accumulating kernels have no fp64 pass"


def test_wide_range_query_in_graph_replays(data):
    gs, torch = _gs()
    docs, (qs, ks, wide) = data
    idx = gs.Index.from_rows(docs, "fp32")
    opts = gs.make_opts("tiled")
    ordinary = qs.subset(np.arange(7, 40))
    k_ord = ks[7:]
    batch = gs.Batch.reserve(idx, qs.n_rows, qs.nnz, 1024)
    ws = idx.workspace(qs.n_rows, opts)
    ids = torch.empty((qs.n_rows, 1024), dtype=torch.int32, device="cuda")
    sc = torch.empty((qs.n_rows, 1024), dtype=torch.float32, device="cuda")
    batch.update(ordinary, k_ord)  # captured without any wide-range query
    graph = gs.Graph(idx, batch, ws, ids, sc, opts)
    for rep, (sub, kk) in enumerate([(qs, ks), (ordinary, k_ord), (qs, ks)]):
        torch.cuda.synchronize()
        batch.update(sub, kk)
        ids.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        n = sub.n_rows
        check_batch("fp32", docs, sub, ids.cpu().numpy()[:n], sc.cpu().numpy()[:n], kk, what="replay %d" % rep)
        d = batch.diagnostics()
        if n == qs.n_rows:
            assert all(d[q, 4] == 2 for q, wd in enumerate(wide) if wd is True), "replay %d" % rep
    graph.close()


def test_bf16_band_overflow_is_an_error_of_the_synchronous_search():
    # 60,000 exact ties at the k-th score: the bf16 band holds every document, more than the
    # band buffer: the batch form flags the row, the synchronous form returns GS_ECAPACITY
    gs, torch = _gs()
    docs = csr([[(0, 1.0)] for _ in range(60_000)], 4)
    qs = csr([[(0, 1.0)], [(1, 1.0)]], 4)
    idx = gs.Index.from_rows(docs, "bf16")
    b = idx.batch(qs, [100, 100], k_max=100)
    idx.search(b, idx.workspace(2))
    torch.cuda.synchronize()
    d = b.diagnostics()
    assert d[0, 3] == 1 and d[1, 3] == 0
    with pytest.raises(gs.GsError) as e:
        idx.search_host(qs, [100, 100], k_max=100)
    assert e.value.code == gs.GS_ECAPACITY
