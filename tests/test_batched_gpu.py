"""Batched search of uneven queries (shared traversal, autotuner, hipGraph), against the oracle.

* The autotuner: every candidate option set (kernel x doc tile x chunk) must give
  the default search's result bit for bit (integer and fixed-point sums do not
  depend on the launch shape), the returned best must be one of the candidates,
  and the outputs it leaves must be the best candidate's.
* The long-tailed batch (lognormal lengths, median 25, up to 250 terms; k mixed
  over {10, 100, 1000}) of 1,024 queries over 1M documents in one shared-traversal
  search: a sample against the oracle, every query of a hipGraph replay bit for
  bit against the direct search.
"""
import numpy as np
import pytest

import oracle
import workload
from parity_rules import check_batch, check_exact_f64, check_exact_int

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


@pytest.fixture(scope="module")
def tune_data():
    return workload.collection(300_000, seed=61), workload.queries_lognormal(64, seed=62)


@pytest.mark.parametrize("precision", ["u8", "fp32"])
def test_autotune_candidates_agree_and_best_is_one_of_them(tune_data, precision):
    gs, torch = _gs()
    docs, qs = tune_data
    ks = workload.k_mix(qs.n_rows, seed=63)
    idx = gs.Index.from_rows(docs, precision)
    b = idx.batch(qs, ks, k_max=1000)
    ws = idx.workspace(qs.n_rows)
    ref_ids, ref_sc = idx.search(b, ws)
    torch.cuda.synchronize()
    ref_ids, ref_sc = ref_ids.cpu().numpy(), ref_sc.cpu().numpy()
    check_batch(precision, docs, qs, ref_ids, ref_sc, ks, what="default")
    best, table, out = idx.autotune(b, ws, reps=1, cache=False, return_outputs=True)
    names = {gs.GS_KERNEL_TILED: "tiled", gs.GS_KERNEL_SHARED: "shared", gs.GS_KERNEL_GROUP: "group"}
    cands = [(c["kernel"], c["tile_docs"], c["chunk"]) for c, _ in table]
    expect_tiles = [8192, 16384] + ([] if precision == "fp32" else [32768])
    assert len(cands) == 2 * len(expect_tiles) * 4 + 3 and len(set(cands)) == len(cands)
    assert (best.kernel, best.tile_docs, best.chunk) in cands
    assert all(t > 0 for _, t in table)
    # the autotuner's outputs are the best candidate's result
    assert np.array_equal(out[0], ref_ids) and np.array_equal(out[1], ref_sc)
    for kern, tile, chunk in cands:
        o = gs.make_opts(names[kern], tile_docs=tile, chunk=chunk)
        ids, sc = idx.search(b, ws, o)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), ref_ids), (kern, tile, chunk)
        assert np.array_equal(sc.cpu().numpy(), ref_sc), (kern, tile, chunk)


def test_autotune_cache_is_keyed_by_index_and_k_max(tune_data):
    gs, torch = _gs()
    docs, qs = tune_data
    sub = qs.subset(np.arange(8))
    idx1 = gs.Index.from_rows(docs, "u8")
    idx2 = gs.Index.from_rows(docs, "u8")
    b1 = idx1.batch(sub, 100, k_max=100)
    b2 = idx2.batch(sub, 100, k_max=100)
    b3 = idx1.batch(sub, 100, k_max=1000)
    r1 = idx1.autotune(b1, reps=1)
    assert idx1.autotune(b1, reps=1) is r1  # cached
    assert idx2.autotune(b2, reps=1) is not r1  # another index
    assert idx1.autotune(b3, reps=1) is not r1  # another k_max


@pytest.fixture(scope="module")
def uneven():
    w = workload.WORKLOADS["mid-1m"]
    docs = workload.make_collection(w)
    qs = workload.queries_lognormal(1024, seed=64)
    return docs, qs, workload.k_mix(qs.n_rows, seed=65)


@pytest.mark.parametrize("precision,kernel", [("u8", "shared"), ("bf16", "shared"), ("u8", "group"),
                                              ("bf16", "group")])
def test_uneven_batch_shared_traversal_and_graph(uneven, precision, kernel):
    gs, torch = _gs()
    docs, qs, ks = uneven
    assert qs.n_rows == 1024 and np.diff(qs.row_ptr).max() <= 250
    idx = gs.Index.from_rows(docs, precision)
    opts = gs.make_opts(kernel)
    b = idx.batch(qs, ks, k_max=1000)
    ws = idx.workspace(qs.n_rows, opts)
    ids, sc = idx.search(b, ws, opts)
    torch.cuda.synchronize()
    assert b.diagnostics()[:, 3].max() == 0
    d_ids, d_sc = ids.cpu().numpy(), sc.cpu().numpy()
    # oracle on a sample that includes the longest queries
    lens = np.diff(qs.row_ptr)
    pick = np.unique(np.r_[np.arange(12), np.argsort(-lens)[:4]])
    sub = qs.subset(pick)
    if precision == "u8":
        rid, rsc = oracle.topk_i64(docs, sub, ks[pick], k_max=1000)
        for i, q in enumerate(pick):
            check_exact_int(d_ids[q], d_sc[q], rid[i], rsc[i], "q%d" % q)
    else:
        rid, rsc = oracle.topk_f64(docs, sub, ks[pick], k_max=1000)
        for i, q in enumerate(pick):
            check_exact_f64(d_ids[q], d_sc[q], rid[i], rsc[i], "q%d" % q)
    # a captured graph of the same search, replayed after unrelated eager work
    gids = torch.full_like(ids, -7)
    gsc = torch.zeros_like(sc)
    graph = gs.Graph(idx, b, ws, gids, gsc, opts)
    scratch = torch.randn(256, 256, device="cuda")
    for rep in range(2):
        scratch = scratch @ scratch.T / 256.0
        torch.cuda.synchronize()
        gids.fill_(-7)
        graph.launch()
        torch.cuda.synchronize()
        assert np.array_equal(gids.cpu().numpy(), d_ids), "replay %d" % rep
        assert np.array_equal(gsc.cpu().numpy(), d_sc), "replay %d" % rep
    graph.close()
