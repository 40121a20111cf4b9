"""Batch reuse (reserve / update) and hipGraph-captured search against direct launches.

Every graph replay is preceded by unrelated eager GPU work and a synchronisation,
and every replay is compared with a direct search of the same queries. The
fixed-point fp32 and the uint8 forms are deterministic, so the comparison is
bit for bit; each direct result is itself checked against the oracle.
"""
import numpy as np
import pytest

import workload
from parity_rules import check_batch

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


@pytest.fixture(scope="module")
def data():
    docs = workload.collection(60_000, seed=71)
    q1 = workload.queries_poisson(24, seed=72)
    q2 = workload.queries_lognormal(24, seed=73)
    return docs, q1, q2


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
@pytest.mark.parametrize("kernel", ["tiled", "shared", "group"])
def test_graph_replays_match_direct_search(data, precision, kernel):
    gs, torch = _gs()
    docs, q1, q2 = data
    idx = gs.Index.from_rows(docs, precision)
    k1 = workload.k_mix(q1.n_rows, seed=5)
    k2 = workload.k_mix(q2.n_rows, seed=6)
    cap_nnz = max(q1.nnz, q2.nnz)
    opts = gs.make_opts(kernel)
    # direct (eager) answers
    direct = {}
    for name, qs, kk in (("q1", q1, k1), ("q2", q2, k2)):
        b = idx.batch(qs, kk, k_max=1000)
        ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
        torch.cuda.synchronize()
        direct[name] = (ids.cpu().numpy(), sc.cpu().numpy())
        check_batch(precision, docs, qs, direct[name][0], direct[name][1], kk, what="direct " + name)
    # one reserved batch, one graph, refilled between replays
    batch = gs.Batch.reserve(idx, q1.n_rows, cap_nnz, 1000)
    ws = idx.workspace(q1.n_rows, opts)
    ids = torch.empty((q1.n_rows, 1000), dtype=torch.int32, device="cuda")
    sc = torch.empty((q1.n_rows, 1000), dtype=gs.SCORE_DTYPES[idx.precision], device="cuda")
    batch.update(q1, k1)
    graph = gs.Graph(idx, batch, ws, ids, sc, opts)
    scratch = torch.randn(512, 512, device="cuda")
    for rep, name in enumerate(["q1", "q2", "q1", "q2", "q2"]):
        scratch = scratch @ scratch.T / 512.0  # unrelated eager work between replays
        torch.cuda.synchronize()
        batch.update(q1 if name == "q1" else q2, k1 if name == "q1" else k2)
        ids.fill_(-7)
        sc.zero_()
        graph.launch()
        torch.cuda.synchronize()
        same = np.array_equal(ids.cpu().numpy(), direct[name][0]) and np.array_equal(sc.cpu().numpy(),
                                                                                      direct[name][1])
        assert same, "replay %d (%s) differs from the direct search" % (rep, name)
    graph.close()


def test_partial_update_pads_with_empty_queries(data):
    gs, torch = _gs()
    docs, q1, _ = data
    idx = gs.Index.from_rows(docs, "u8")
    batch = gs.Batch.reserve(idx, 10, q1.nnz, 100)
    sub = q1.subset(np.arange(4))
    batch.update(sub, 100)
    ids, sc = idx.search(batch, idx.workspace(10))
    torch.cuda.synchronize()
    ids, sc = ids.cpu().numpy(), sc.cpu().numpy()
    check_batch("u8", docs, sub, ids[:4], sc[:4], 100, what="partial")
    assert np.all(ids[4:] == -1) and np.all(sc[4:] == 0)
    with pytest.raises(gs.GsError):
        batch.update(q1, 100)  # 24 queries do not fit a capacity of 10


def test_graph_replay_after_a_refill_with_tiny_products(data):
    # fixed point: products of 1e-30 weights round to 0 units (far below the k-th scores, so the
    # wide-range check leaves the queries alone). A graph captured on a batch without them and
    # replayed after a refill with them must give the direct search's answer, bit for bit.
    gs, torch = _gs()
    docs, q1, q2 = data
    q1_terms = set(q1.terms.tolist())
    t_small = next(int(t) for t in q2.row(0)[0] if int(t) not in q1_terms)
    w = docs.weights.copy()
    hits = np.flatnonzero(docs.terms == t_small)[:50]
    w[hits] = np.float32(1e-30)
    docs_s = workload.SparseRows(docs.row_ptr, docs.terms, w, docs.vocab)
    idx = gs.Index.from_rows(docs_s, "fp32")
    opts = gs.make_opts("tiled")
    k1 = np.full(q1.n_rows, 100, np.int32)
    k2 = np.full(q2.n_rows, 100, np.int32)
    direct = {}
    for name, qs, kk in (("q1", q1, k1), ("q2", q2, k2)):
        b = idx.batch(qs, kk, k_max=100)
        ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
        torch.cuda.synchronize()
        direct[name] = (ids.cpu().numpy(), sc.cpu().numpy())
        check_batch("fp32", docs_s, qs, direct[name][0], direct[name][1], kk, what="direct " + name)
    batch = gs.Batch.reserve(idx, q1.n_rows, max(q1.nnz, q2.nnz), 100)
    ws = idx.workspace(q1.n_rows, opts)
    ids = torch.empty((q1.n_rows, 100), dtype=torch.int32, device="cuda")
    sc = torch.empty((q1.n_rows, 100), dtype=torch.float32, device="cuda")
    batch.update(q1, k1)
    graph = gs.Graph(idx, batch, ws, ids, sc, opts)
    for name in ["q1", "q2", "q1"]:
        torch.cuda.synchronize()
        batch.update(q1 if name == "q1" else q2, k1 if name == "q1" else k2)
        ids.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), direct[name][0]), name
        assert np.array_equal(sc.cpu().numpy(), direct[name][1]), name
    graph.close()


def test_batch_freed_after_its_index(data):
    # a batch keeps its own device memory: freeing it after its index must not touch the index
    gs, torch = _gs()
    docs, q1, _ = data
    idx = gs.Index.from_rows(docs, "u8")
    b = idx.batch(q1, 10)
    ids, sc = idx.search(b, idx.workspace(q1.n_rows))
    torch.cuda.synchronize()
    idx.close()
    b.close()
    idx2 = gs.Index.from_rows(docs, "u8")
    b2 = idx2.batch(q1, 10)
    ids2, sc2 = idx2.search(b2, idx2.workspace(q1.n_rows))
    torch.cuda.synchronize()
    assert np.array_equal(ids.cpu().numpy(), ids2.cpu().numpy())
    check_batch("u8", docs, q1, ids2.cpu().numpy(), sc2.cpu().numpy(), 10, what="after free")
    b2.close()
    idx2.close()


def test_atomic_kernel_needs_the_doc_ids(data):
    gs, torch = _gs()
    docs, q1, _ = data
    idx = gs.Index.from_rows(docs, "fp32")
    with pytest.raises(gs.GsError) as e:
        idx.search(idx.batch(q1, 10), idx.workspace(4), gs.make_opts("atomic"))
    assert e.value.code == gs.GS_EUNSUPPORTED
    full = gs.Index.from_rows(docs, "fp32", keep_doc_ids=True)
    assert full.info().device_bytes - idx.info().device_bytes == 4 * full.info().padded_nnz
