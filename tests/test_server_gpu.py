"""The continuous-batching request loop: results alone vs in a concurrent mix, memory admission, errors."""
import threading

import numpy as np
import pytest

import oracle
import workload
from parity_rules import check_exact_int, check_fp32

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


@pytest.fixture(scope="module")
def data():
    docs = workload.collection(50_000, seed=81)
    qs = workload.queries_lognormal(96, seed=82)
    k = workload.k_mix(96, seed=83)
    return docs, qs, k


@pytest.mark.parametrize("kernel", ["tiled", "shared"])
@pytest.mark.parametrize("precision", ["u8", "fp32"])
def test_results_alone_equal_results_in_the_mix(data, precision, kernel):
    gs, _ = _gs()
    docs, qs, k = data
    idx = gs.Index.from_rows(docs, precision)
    srv = gs.Server(idx, max_batch=8, n_slots=3, k_max=1000, opts=gs.make_opts(kernel))
    # alone: one request at a time
    alone = []
    for q in range(12):
        t, w = qs.row(q)
        alone.append(srv.wait(srv.submit(t, w, int(k[q])), int(k[q]))[:2])
    # in the mix: four threads submit all 96 queries at once
    tickets = {}
    lock = threading.Lock()

    def submitter(lo, hi):
        for q in range(lo, hi):
            t, w = qs.row(q)
            tk = srv.submit(t, w, int(k[q]))
            with lock:
                tickets[q] = tk

    th = [threading.Thread(target=submitter, args=(i * 24, (i + 1) * 24)) for i in range(4)]
    [x.start() for x in th]
    [x.join() for x in th]
    mixed = {q: srv.wait(tickets[q], int(k[q])) for q in range(96)}
    st = srv.stats()
    assert st["completed"] == 108 and st["mean_batch"] > 1.0  # requests really shared device steps
    for q in range(12):
        same = np.array_equal(alone[q][0], mixed[q][0]) and np.array_equal(alone[q][1], mixed[q][1])
        assert same, "query %d differs alone vs in the mix" % q
    # and the mix is right
    sample = qs.subset(np.arange(16))
    if precision == "u8":
        rid, rsc = oracle.topk_i64(docs, sample, k[:16], k_max=1000)
        for q in range(16):
            kq = int(k[q])
            check_exact_int(mixed[q][0], mixed[q][1], rid[q][:kq], rsc[q][:kq], what="served q%d" % q)
    else:
        rid, rsc = oracle.topk_f64(docs, sample, k[:16], k_max=1000)
        for q in range(16):
            t, w = qs.row(q)
            kq = int(k[q])
            ids = np.concatenate([mixed[q][0], -np.ones(1000 - kq, np.int32)])
            sc = np.concatenate([mixed[q][1], np.zeros(1000 - kq, np.float32)])
            check_fp32(docs, t, w, ids, sc, rid[q], rsc[q], kq, what="served q%d" % q)
    assert all(mixed[q][2] > 0 for q in range(96))
    srv.close()


def test_memory_budget_bounds_the_slots(data):
    gs, _ = _gs()
    docs, qs, k = data
    idx = gs.Index.from_rows(docs, "u8")
    one = idx.workspace_bytes(8)
    srv = gs.Server(idx, max_batch=8, n_slots=6, k_max=100, memory_budget=2 * one + one // 2)
    assert srv.stats()["n_slots"] == 2
    srv.close()
    with pytest.raises(gs.GsError) as e:
        gs.Server(idx, max_batch=8, n_slots=2, k_max=100, memory_budget=one // 2)
    assert e.value.code == gs.GS_ECAPACITY


def test_bad_requests_are_rejected(data):
    gs, _ = _gs()
    docs, qs, k = data
    idx = gs.Index.from_rows(docs, "u8")
    srv = gs.Server(idx, max_batch=4, n_slots=1, k_max=100)
    with pytest.raises(gs.GsError):
        srv.submit([1, 1], [1.0, 2.0], 10)  # duplicate term
    with pytest.raises(gs.GsError):
        srv.submit([1], [1.0], 101)  # k above k_max
    with pytest.raises(gs.GsError):
        srv.submit([40000], [1.0], 10)  # term outside the vocabulary
    t = srv.submit([], [], 5)  # empty query: score-0 docs by id
    ids, sc, _ = srv.wait(t, 5)
    assert ids.tolist() == [0, 1, 2, 3, 4] and np.all(sc == 0)
    srv.close()
