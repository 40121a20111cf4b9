"""Fused candidate filtering against the full row scan.

With the doc-tiled kernels and searches of at least 32 queries, every 8th doc
tile (every 4th for k_max above 1024) is scored first; a lower bound of each query's k-th composite key comes from
those tiles, the other tiles append every composite at or above it while they
are scored, and the filter scans only the seed tiles' scores. The answer must
be the one of the full row scan bit for bit (integer and fixed-point sums do not
depend on order), including the fallbacks: no bound, too many appended, or a
refinement of the threshold (massive ties).
"""
import numpy as np
import pytest

import oracle
import workload
from helpers import random_rows
from parity_rules import check_batch

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


@pytest.fixture(scope="module")
def data():
    docs = workload.collection(300_000, seed=61)
    qs = workload.queries_lognormal(80, seed=62)
    return docs, qs


def _search(gs, torch, idx, qs, k, k_max, kernel, fused, tile_docs=0):
    opts = gs.make_opts(kernel, tile_docs=tile_docs, fused_filter=fused)
    b = idx.batch(qs, k, k_max)
    ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
    torch.cuda.synchronize()
    diag = b.diagnostics()
    assert np.all(diag[:, 3] == 0), "candidate overflow"
    return ids.cpu().numpy(), sc.cpu().numpy(), diag


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
@pytest.mark.parametrize("kernel", ["tiled", "shared", "group"])
def test_fused_equals_row_scan(data, precision, kernel):
    gs, torch = _gs()
    docs, qs = data
    idx = gs.Index.from_rows(docs, precision)
    k = workload.k_mix(qs.n_rows, seed=63)
    a = _search(gs, torch, idx, qs, k, 1000, kernel, True)
    b = _search(gs, torch, idx, qs, k, 1000, kernel, False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # the fused path really ran: its candidate sets differ from the row scan's
    assert np.any(a[2][:, 0] != b[2][:, 0])
    sub = qs.subset(np.arange(6))
    check_batch(precision, docs, sub, a[0][:6], a[1][:6], k[:6], what="fused")
    idx.close()


@pytest.mark.parametrize("tile_docs", [8192, 16384, 32768])
def test_fused_tiles_and_large_k(data, tile_docs):
    # k up to 2000 (seed stride 4 above 1024) and every doc tile size of the uint8 index
    gs, torch = _gs()
    docs, qs = data
    idx = gs.Index.from_rows(docs, "u8")
    k = np.where(np.arange(qs.n_rows) % 2 == 0, 2000, 7).astype(np.int32)
    for kernel in ("tiled", "shared") + (("group",) if tile_docs == 8192 else ()):
        a = _search(gs, torch, idx, qs, k, 2000, kernel, True, tile_docs)
        b = _search(gs, torch, idx, qs, k, 2000, kernel, False, tile_docs)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), kernel
    rid, rsc = oracle.topk_i64(docs, qs.subset(np.arange(4)), k[:4], k_max=2000)
    for q in range(4):
        assert np.array_equal(a[0][q], rid[q]) and np.array_equal(a[1][q].astype(np.int64), rsc[q])
    idx.close()


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_fused_fallback_on_massive_ties(precision):
    # all weights 1: scores are shared-term counts, huge exact ties at the k-th score. The
    # appended candidates pass their cap or the threshold needs refining: the row scan decides.
    gs, torch = _gs()
    rng = np.random.default_rng(64)
    docs = random_rows(rng, 300_000, 60, 1, 8, weight_fn=lambda r, n: np.ones(n))
    qs = random_rows(rng, 40, 60, 1, 6, weight_fn=lambda r, n: np.ones(n))
    idx = gs.Index.from_rows(docs, precision)
    for kernel in ("tiled", "shared", "group"):
        a = _search(gs, torch, idx, qs, 1000, 1000, kernel, True)
        b = _search(gs, torch, idx, qs, 1000, 1000, kernel, False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), kernel
    sub = qs.subset(np.arange(6))
    check_batch(precision, docs, sub, a[0][:6], a[1][:6], 1000, what="ties")
    idx.close()


def test_fused_bf16_band_pass_scores_the_other_tiles():
    # all weights 1 and one-term queries: every doc of the term ties at the k-th score, among
    # the seed tiles too, so the seed bound sits on that score and the bf16 error band below
    # the k-th approximate score reaches under it. A fused query then has no rows for its other
    # tiles: they are scored for the band pass (diagnostics word 4 = 3), and the result must
    # equal the row scan's and the oracle's
    gs, torch = _gs()
    rng = np.random.default_rng(66)
    docs = random_rows(rng, 300_000, 100, 1, 8, weight_fn=lambda r, n: np.ones(n))
    qs = random_rows(rng, 40, 100, 1, 1, weight_fn=lambda r, n: np.ones(n))
    idx = gs.Index.from_rows(docs, "bf16")
    for kernel in ("tiled", "shared", "group"):
        a = _search(gs, torch, idx, qs, 10, 10, kernel, True)
        b = _search(gs, torch, idx, qs, 10, 10, kernel, False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), kernel
        assert np.any(a[2][:, 4] == 3), "%s: no band pass took the other tiles' rows" % kernel
        assert np.all(b[2][:, 4] != 3), kernel
    check_batch("bf16", docs, qs.subset(np.arange(6)), a[0][:6], a[1][:6], 10, what="bf16 band rows")
    idx.close()


def test_fused_graph_replays(data):
    gs, torch = _gs()
    docs, qs = data
    idx = gs.Index.from_rows(docs, "fp32")
    q1, q2 = qs.subset(np.arange(0, 40)), qs.subset(np.arange(40, 80))
    k = np.full(40, 1000, np.int32)
    opts = gs.make_opts("shared")
    direct = []
    for qq in (q1, q2):
        ids, sc, _ = _search(gs, torch, idx, qq, k, 1000, "shared", False)
        direct.append((ids, sc))
    batch = gs.Batch.reserve(idx, 40, max(q1.nnz, q2.nnz), 1000)
    ws = idx.workspace(40, opts)
    ids = torch.empty((40, 1000), dtype=torch.int32, device="cuda")
    sc = torch.empty((40, 1000), dtype=torch.float32, device="cuda")
    batch.update(q1, k)
    graph = gs.Graph(idx, batch, ws, ids, sc, opts)
    for rep in [0, 1, 0, 1]:
        torch.cuda.synchronize()
        batch.update(q1 if rep == 0 else q2, k)
        ids.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), direct[rep][0]) and np.array_equal(sc.cpu().numpy(), direct[rep][1])
    graph.close()
    idx.close()


@pytest.mark.parametrize("n_terms", [(1, 8), (1, 20)])
def test_fused_bf16_band_below_the_candidates(n_terms):
    # dyadic weights (exact in bf16) give many equal scores near the k-th: the bf16 error band
    # then reaches below the fused candidates of some queries, whose rows are scored again
    # before the band pass; fallbacks and fused queries must all equal the row scan
    gs, torch = _gs()
    rng = np.random.default_rng(65 + n_terms[1])
    dy = lambda r, n: r.integers(1, 13, n) / 4.0
    docs = random_rows(rng, 300_000, 200, n_terms[0], n_terms[1], weight_fn=dy)
    qs = random_rows(rng, 40, 200, 3, 12, weight_fn=dy)
    idx = gs.Index.from_rows(docs, "bf16")
    for kernel in ("tiled", "shared", "group"):
        a = _search(gs, torch, idx, qs, 1000, 1000, kernel, True)
        b = _search(gs, torch, idx, qs, 1000, 1000, kernel, False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), kernel
    check_batch("bf16", docs, qs.subset(np.arange(6)), a[0][:6], a[1][:6], 1000, what="bf16 band")
    idx.close()
