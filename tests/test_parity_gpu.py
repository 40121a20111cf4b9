"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by element.

Sizes: the 10K-doc workload and synthetic instances spanning several doc tiles
with a ragged tail, the 1M-doc workload on a query subset, and edge cases
(empty query, k > N, k = 0, longest queries, exact ties, queries matching fewer
than k documents).
"""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from helpers import csr, dense_terms, dyadic, mixed_density_collection, random_rows
from parity_rules import check_batch, check_exact_f64, check_exact_int

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KERNELS = ["tiled", "atomic", "docpar", "shared", "group"]


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs


def _run(gs, docs, queries, k, precision, kernel="tiled", tile_docs=0, chunk=0, query_tile=0, k_max=None):
    idx = gs.Index.from_rows(docs, precision, keep_forward=(kernel == "docpar"),
                              keep_doc_ids=(kernel == "atomic"))
    b = idx.batch(queries, k, k_max)
    opts = gs.make_opts(kernel, query_tile=query_tile, tile_docs=tile_docs, chunk=chunk)
    ws = idx.workspace(max(1, min(queries.n_rows, 64)), opts)
    ids, sc = idx.search(b, ws, opts)
    import torch
    torch.cuda.synchronize()
    diag = b.diagnostics()
    assert np.all(diag[:, 3] == 0), "candidate overflow"
    return ids.cpu().numpy(), sc.cpu().numpy(), diag


@pytest.fixture(scope="module")
def tiny():
    w = workload.WORKLOADS["tiny-10k"]
    return workload.make_collection(w), workload.make_queries(w)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "u8"])
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("k", [10, 100])
def test_tiny_workload(tiny, precision, kernel, k):
    gs = _gs()
    docs, qs = tiny
    ids, sc, _ = _run(gs, docs, qs, k, precision, kernel)
    check_batch(precision, docs, qs, ids, sc, k, what="tiny %s %s k%d" % (precision, kernel, k))


@pytest.mark.parametrize("precision", ["fp32", "bf16", "u8"])
def test_hand_worked_example(precision):
    gs = _gs()
    g = json.load(open(os.path.join(GOLDEN, "tiny_example.json")))
    docs, qs = csr(g["docs"], g["vocab"]), csr(g["queries"], g["vocab"])
    for kernel in KERNELS:
        ids, sc, _ = _run(gs, docs, qs, g["k"], precision, kernel)
        exp = g["expected_i64"] if precision == "u8" else g["expected_f64"]
        ok_ids = ids.tolist() == exp["ids"]
        ok_sc = np.array_equal(sc.astype(np.float64), np.asarray(exp["scores"], np.float64))
        assert ok_ids and ok_sc, kernel


@pytest.mark.parametrize("precision,tile_docs", [("fp32", 8192), ("fp32", 16384), ("u8", 8192), ("u8", 16384),
                                                 ("u8", 32768), ("bf16", 8192), ("bf16", 16384),
                                                 ("bf16", 32768)])
@pytest.mark.parametrize("chunk", [64, 256, 1024])
def test_dyadic_weights_are_exact_across_tiles(precision, tile_docs, chunk):
    # multiples of 1/16: every sum is exact, so fp32 scores must equal the fp64 oracle bit for bit
    gs = _gs()
    rng = np.random.default_rng(tile_docs + chunk)
    docs = random_rows(rng, 41_000, 300, 1, 25, weight_fn=dyadic)
    qs = random_rows(rng, 12, 300, 1, 40, weight_fn=dyadic)
    if precision == "u8":
        rid, rsc = oracle.topk_i64(docs, qs, 300)
    else:
        rid, rsc = oracle.topk_f64(docs, qs, 300)
    kernels = ("tiled", "atomic", "shared") if precision == "fp32" else ("tiled", "shared")
    if tile_docs == 8192 and chunk >= 256:
        kernels = kernels + ("group",)  # the group kernel: 8192-doc tiles, chunks of 256+
    for kernel in kernels:
        ids, sc, _ = _run(gs, docs, qs, 300, precision, kernel, tile_docs=tile_docs, chunk=chunk)
        for q in range(qs.n_rows):
            if precision == "u8":
                check_exact_int(ids[q], sc[q], rid[q], rsc[q], "%s q%d" % (kernel, q))
            else:
                check_exact_f64(ids[q], sc[q], rid[q], rsc[q], "%s q%d" % (kernel, q))


def test_fp32_tiles_reject_32768_docs():
    # 32768 docs of 64-bit accumulators do not fit one CU's LDS
    gs = _gs()
    docs = random_rows(np.random.default_rng(2), 100, 20, 1, 5)
    idx = gs.Index.from_rows(docs, "fp32")
    with pytest.raises(gs.GsError) as e:
        idx.workspace_bytes(1, gs.make_opts("tiled", tile_docs=32768))
    assert e.value.code == gs.GS_EUNSUPPORTED


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
def test_all_ones_weights_massive_ties(precision):
    # scores are shared-term counts: thousands of exact ties at the k-th score, decided by doc id
    gs = _gs()
    rng = np.random.default_rng(5)
    docs = random_rows(rng, 30_000, 40, 1, 10, weight_fn=lambda r, n: np.ones(n))
    qs = random_rows(rng, 6, 40, 1, 8, weight_fn=lambda r, n: np.ones(n))
    for kernel in KERNELS:
        ids, sc, diag = _run(gs, docs, qs, 1000, precision, kernel)
        check_batch(precision, docs, qs, ids, sc, 1000, what="ones %s" % kernel)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "u8"])
def test_edge_cases(precision):
    gs = _gs()
    rng = np.random.default_rng(11)
    V = 30522
    docs = workload.collection(20_000, seed=99)
    long_q = [(int(t), float(w)) for t, w in zip(np.sort(rng.choice(V, 256, replace=False)),
                                                 np.log1p(rng.lognormal(0, 0.8, 256)))]
    rare = int(np.argmin(np.where(np.bincount(docs.terms, minlength=V) > 0,
                                  np.bincount(docs.terms, minlength=V), 1 << 30)))
    rows = [
        [],                        # empty query: all scores 0, ids ascending
        long_q,                    # the longest allowed query
        [(rare, 1.0)],             # matches very few docs: the answer is filled by doc id
        [(int(docs.terms[0]), 2.0), (int(docs.terms[1]), 0.5)],
    ]
    qs = csr(rows, V)
    k = np.array([7, 1000, 1000, 0], np.int32)
    for kernel in KERNELS:
        ids, sc, diag = _run(gs, docs, qs, k, precision, kernel, k_max=1000)
        check_batch(precision, docs, qs, ids, sc, k, what="edge %s" % kernel)
        assert np.all(ids[3] == -1)


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_k_beyond_collection_and_tiny_collections(precision):
    gs = _gs()
    rng = np.random.default_rng(12)
    for n in (1, 5, 63, 64, 65, 3000):
        docs = random_rows(rng, n, 20, 1, 6)
        qs = random_rows(rng, 3, 20, 1, 5)
        for kernel in KERNELS:
            ids, sc, _ = _run(gs, docs, qs, [n + 3, max(1, n // 2), n], precision, kernel, k_max=n + 3)
            check_batch(precision, docs, qs, ids, sc, [n + 3, max(1, n // 2), n], what="n%d %s" % (n, kernel))


@pytest.mark.parametrize("precision", ["u8", "fp32"])
def test_query_tiling_and_block_order_do_not_change_results(tiny, precision):
    # integer sums (uint8 impacts, and the fixed-point fp32 accumulators) do not depend on update order
    gs = _gs()
    docs, qs = tiny
    a, sa, _ = _run(gs, docs, qs, 100, precision, "tiled", query_tile=3)
    b, sb, _ = _run(gs, docs, qs, 100, precision, "tiled", query_tile=0)
    c, sc, _ = _run(gs, docs, qs, 100, precision, "shared", query_tile=5)
    same = all(np.array_equal(x, y) for x, y in ((a, b), (sa, sb), (a, c), (sa, sc)))
    assert same


def test_host_csr_entry_point_matches_prepared_batch(tiny):
    # integer path: accumulation is order-independent, so two runs must agree bit for bit
    gs = _gs()
    docs, qs = tiny
    idx = gs.Index.from_rows(docs, "u8")
    ids, sc = idx.search_host(qs, 100)
    ids2, sc2 = idx.search(idx.batch(qs, 100))
    same = np.array_equal(ids.cpu().numpy(), ids2.cpu().numpy()) and np.array_equal(sc.cpu().numpy(),
                                                                                     sc2.cpu().numpy())
    assert same


def test_search_errors_are_reported():
    gs = _gs()
    import torch
    docs = random_rows(np.random.default_rng(1), 100, 20, 1, 5)
    idx = gs.Index.from_rows(docs, "fp32")
    qs = csr([[(1, 1.0)]], 20)
    b = idx.batch(qs, 5)
    tiny_ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(gs.GsError) as e:
        idx.search(b, tiny_ws)
    assert e.value.code == gs.GS_ECAPACITY
    with pytest.raises(gs.GsError) as e:
        idx.search(b, opts=gs.make_opts("docpar"))
    assert e.value.code == gs.GS_EUNSUPPORTED
    with pytest.raises(gs.GsError):
        idx.batch(csr([[(1, 1.0), (1, 2.0)]], 20), 5)
    with pytest.raises(gs.GsError):
        idx.batch(qs, [gs.GS_MAX_K + 1])


@pytest.fixture(scope="module")
def mid():
    w = workload.WORKLOADS["mid-1m"]
    return workload.make_collection(w), workload.make_queries(w, n=48)


@pytest.mark.parametrize("precision,kernel", [("fp32", "tiled"), ("fp32", "atomic"), ("fp32", "docpar"),
                                              ("fp32", "shared"), ("u8", "tiled"), ("u8", "shared"),
                                              ("bf16", "tiled"), ("bf16", "shared"), ("fp32", "group"),
                                              ("u8", "group"), ("bf16", "group")])
def test_mid_scale_top1000(mid, precision, kernel):
    gs = _gs()
    docs, qs = mid
    ids, sc, diag = _run(gs, docs, qs, 1000, precision, kernel)
    check_batch(precision, docs, qs, ids, sc, 1000, what="1M %s %s" % (precision, kernel))


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_refinement_rounds_resolve_massive_exact_ties(precision):
    # every document holds term 0 with weight 1 and the query is {0: 1}: all 150,000 docs tie
    # exactly, the first digit bucket overflows the candidate buffer and the answer is decided by
    # doc id through the refinement rounds
    gs = _gs()
    rng = np.random.default_rng(21)
    rows = []
    for _ in range(150_000):
        extra = rng.choice(np.arange(1, 24), size=int(rng.integers(0, 3)), replace=False)
        rows.append([(0, 1.0)] + [(int(e), float(rng.integers(1, 3))) for e in sorted(extra)])
    docs = csr(rows, 24)
    qs = csr([[(0, 1.0)], [(0, 1.0), (5, 1.0)], [(0, 0.5)]], 24)
    k = [1000, 4000, 7]
    ids, sc, diag = _run(gs, docs, qs, k, precision, "tiled", k_max=4096)
    assert diag[0, 1] > 0, "the all-tied query needed no refinement round"
    check_batch(precision, docs, qs, ids, sc, k, what="refine " + precision)


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_fused_fallback_then_refinement(precision):
    # 33 queries turn fused filtering on (seed stride 4 for k_max 2048 over 19 tiles). The
    # all-tied query appends every non-seed doc, passes the cap and falls back: its other
    # tiles are scored and counted again, its selection is redone from the complete
    # histogram, and the tie at the k-th score needs refinement rounds.
    gs = _gs()
    rng = np.random.default_rng(21)
    rows = []
    for _ in range(150_000):
        extra = rng.choice(np.arange(1, 24), size=int(rng.integers(0, 3)), replace=False)
        rows.append([(0, 1.0)] + [(int(e), float(rng.integers(1, 3))) for e in sorted(extra)])
    docs = csr(rows, 24)
    base = [[(0, 1.0)], [(0, 1.0), (5, 1.0)], [(0, 0.5)]]
    qs = csr(base * 11, 24)
    k = [1000, 2000, 7] * 11
    first = None
    for kernel in ("tiled", "shared"):
        ids, sc, diag = _run(gs, docs, qs, k, precision, kernel, k_max=2048)
        assert diag[0, 1] > 0, "the all-tied query needed no refinement round"
        for c in range(1, 11):  # every copy of a query gets the same answer
            assert np.array_equal(ids[3 * c:3 * c + 3], ids[:3]) and np.array_equal(sc[3 * c:3 * c + 3], sc[:3])
        if first is None:
            first = (ids[:3], sc[:3])
            check_batch(precision, docs, qs.subset(np.arange(3)), ids[:3], sc[:3], k[:3],
                        what="fused fallback " + precision)
        else:
            assert np.array_equal(ids[:3], first[0]) and np.array_equal(sc[:3], first[1]), kernel


def test_bf16_band_beyond_capacity_is_flagged_not_wrong():
    # with the same exact ties the bf16 rescoring band holds every document: beyond the
    # candidate buffer, so the row must be flagged as overflowed
    gs = _gs()
    rows = [[(0, 1.0)] for _ in range(60_000)]
    docs = csr(rows, 4)
    qs = csr([[(0, 1.0)]], 4)
    idx = gs.Index.from_rows(docs, "bf16")
    b = idx.batch(qs, [100], k_max=100)
    idx.search(b, idx.workspace(1))
    import torch
    torch.cuda.synchronize()
    assert b.diagnostics()[0, 3] == 1


@pytest.fixture(scope="module")
def full():
    w = workload.WORKLOADS["full-8.8m"]
    return workload.make_collection(w), workload.make_queries(w)


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
def test_full_scale_sampled(full, precision):
    # the benchmark's configuration: 8.8M docs, all 500 queries in one launch, top-1000, with the
    # per-query (tiled) and the shared-traversal kernel. The oracle checks a sample of queries
    # completely and every returned score of every 25th query one by one; the two kernels must
    # agree bit for bit on all 500 queries (integer and fixed-point sums do not depend on order).
    gs = _gs()
    import torch
    docs, qs = full
    idx = gs.Index.from_rows(docs, precision)
    got = {}
    for kernel in ("tiled", "shared", "group"):
        opts = gs.make_opts(kernel)
        b = idx.batch(qs, 1000)
        ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
        torch.cuda.synchronize()
        assert b.diagnostics()[:, 3].max() == 0
        got[kernel] = (ids.cpu().numpy(), sc.cpu().numpy())
        del ids, sc, b
        torch.cuda.empty_cache()
    ids, sc = got["tiled"]
    assert np.array_equal(ids, got["shared"][0]) and np.array_equal(sc, got["shared"][1]), "tiled vs shared"
    assert np.array_equal(ids, got["group"][0]) and np.array_equal(sc, got["group"][1]), "tiled vs group"
    sample = qs.subset(np.arange(6))
    check_batch(precision, docs, sample, ids[:6], sc[:6], 1000, n_threads=0, what="8.8M " + precision)
    for q in range(0, qs.n_rows, 25):  # every 25th query: returned scores are the exact scores of those docs
        t, w = qs.row(q)
        f, i = oracle.pair_scores(docs, t, w, ids[q])
        if precision == "u8":
            assert np.array_equal(sc[q].astype(np.int64), i)
        elif precision == "bf16":
            assert np.array_equal(sc[q], f)
        else:
            assert np.max(np.abs(sc[q] - f) / f) < 1e-5
        assert np.all(np.diff(sc[q]) <= 0) and np.unique(ids[q]).shape[0] == 1000
    idx.close()


@pytest.mark.parametrize("kernel", ["tiled", "shared"])
def test_bf16_fixed_point_headroom(kernel):
    # bf16 scores are summed in 32-bit fixed point, scaled per query so that the largest possible
    # sum (every query term at its largest stored weight) stays below 2^32 units. Docs that reach
    # that largest sum exactly must not wrap around: they are the top of the answer, and the
    # rescored result must equal the fp64 oracle's.
    gs = _gs()
    rng = np.random.default_rng(21)
    V = 2000
    q_terms = np.sort(rng.choice(V, 250, replace=False)).astype(np.int32)
    rows = []
    for d in range(20_000):
        if d % 997 == 0:  # every query term at 3.0, the largest weight of each of its lists
            rows.append([(int(t), 3.0) for t in q_terms])
        else:
            n = int(rng.integers(5, 60))
            t = np.sort(rng.choice(V, n, replace=False))
            rows.append([(int(a), float(w)) for a, w in zip(t, rng.uniform(0.01, 2.9, n))])
    docs = csr(rows, V)
    qs = csr([[(int(t), 3.0) for t in q_terms], [(int(t), float(w)) for t, w in zip(q_terms, rng.uniform(0.5, 3.0, 250))]], V)
    rid, rsc = oracle.topk_f64(docs, qs, 100)
    full = list(range(0, 20_000, 997))
    assert rsc[0, 0] == 250 * 9.0 and sorted(rid[0][:len(full)].tolist()) == full
    assert sorted(rid[1][:len(full)].tolist()) == full
    ids, sc, _ = _run(gs, docs, qs, 100, "bf16", kernel, tile_docs=32768)
    for q in range(qs.n_rows):
        check_exact_f64(ids[q], sc[q], rid[q], rsc[q], "headroom q%d" % q)


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
def test_byte_doc_ids_of_dense_terms(precision):
    # dense and 2-byte lists mixed in one query, segments that start and end inside a
    # 64-posting block, a block across a tile boundary, a zero-weight dense term (the byte
    # form is read by the per-query kernel with fp32 and bf16 weights; the other cases
    # check the same instances on the 2-byte form)
    gs = _gs()
    rng = np.random.default_rng(77)
    docs = mixed_density_collection(rng)
    qrows = [[(0, 1.0), (1, 0.5), (2, 2.0)], [(3, 1.0), (4, 0.25), (5, 1.5)],
             [(t, float(dyadic(rng, 1)[0])) for t in range(8)] + [(11, 1.0), (200, 0.5)],
             [(6, 3.0)], [(0, 0.0), (3, 1.0)], [(6, 1.0), (7, 1.0)]]
    for _ in range(6):
        ts = sorted(set(rng.choice(8, size=3, replace=False).tolist()) | set(rng.choice(np.arange(10, 320), size=4).tolist()))
        qrows.append([(int(t), float(w)) for t, w in zip(ts, dyadic(rng, len(ts)))])
    qs = csr(qrows, docs.vocab)
    k = 200
    if precision == "u8":
        rid, rsc = oracle.topk_i64(docs, qs, k)
    else:
        rid, rsc = oracle.topk_f64(docs, qs, k)
    expect_dense = dense_terms(docs)
    assert list(np.flatnonzero(expect_dense)) == [0, 1, 2, 6]
    shapes = [(8192, 64), (16384, 1024)] + ([(32768, 256)] if precision != "fp32" else [(8192, 256)])
    for kernel in ("tiled", "shared"):
        for tile_docs, chunk in shapes:
            idx = gs.Index.from_rows(docs, precision)
            assert np.array_equal(idx.dense_terms(), expect_dense)
            assert idx.info().n_dense_terms == int(expect_dense.sum())
            short = np.zeros(docs.vocab - 1, dtype=np.uint8)
            assert gs.lib.gs_index_dense_terms(idx.handle, short.ctypes.data, docs.vocab - 1) == -1
            idx.close()
            ids, sc, _ = _run(gs, docs, qs, k, precision, kernel, tile_docs=tile_docs, chunk=chunk)
            for q in range(qs.n_rows):
                what = "%s tile %d chunk %d q%d" % (kernel, tile_docs, chunk, q)
                if precision == "u8":
                    check_exact_int(ids[q], sc[q], rid[q], rsc[q], what)
                else:
                    check_exact_f64(ids[q], sc[q], rid[q], rsc[q], what)
