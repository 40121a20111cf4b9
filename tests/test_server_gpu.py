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


@pytest.mark.parametrize("kernel", ["tiled", "shared", "group"])
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


def test_memory_budget_bounds_the_queries_in_flight(data):
    # admission by memory: the arena holds as many query rows (score array + selection scratch)
    # as the budget allows, whatever n_slots x max_batch would take
    gs, _ = _gs()
    docs, qs, k = data
    idx = gs.Index.from_rows(docs, "u8")
    budget = idx.workspace_bytes(10) + idx.workspace_bytes(1) // 2
    srv = gs.Server(idx, max_batch=8, n_slots=4, k_max=1000, memory_budget=budget)
    st = srv.stats()
    assert st["arena_rows"] == 10 and st["arena_bytes"] <= budget
    tickets = []
    for q in range(96):
        t, w = qs.row(q)
        tickets.append(srv.submit(t, w, int(k[q])))
    got = [srv.wait(tickets[q], int(k[q])) for q in range(96)]
    st = srv.stats()
    assert 1 <= st["max_in_flight"] <= 10 and st["completed"] == 96
    rid, rsc = oracle.topk_i64(docs, qs.subset(np.arange(16)), k[:16], k_max=1000)
    for q in range(16):
        kq = int(k[q])
        check_exact_int(got[q][0], got[q][1], rid[q][:kq], rsc[q][:kq], what="budgeted q%d" % q)
    srv.close()
    with pytest.raises(gs.GsError) as e:
        gs.Server(idx, max_batch=8, n_slots=2, k_max=100, memory_budget=idx.workspace_bytes(1) // 2)
    assert e.value.code == gs.GS_ECAPACITY


def test_poll_and_single_collection(data):
    gs, _ = _gs()
    docs, qs, k = data
    idx = gs.Index.from_rows(docs, "u8")
    srv = gs.Server(idx, max_batch=4, n_slots=2, k_max=100)
    t, w = qs.row(0)
    tk = srv.submit(t, w, 100)
    res = None
    for _ in range(200000):
        res = srv.poll(tk, 100)
        if res is not None:
            break
    assert res is not None
    ref = srv.wait(srv.submit(t, w, 100), 100)
    assert np.array_equal(res[0], ref[0]) and np.array_equal(res[1], ref[1])
    with pytest.raises(gs.GsError) as e:  # a ticket is collected once
        srv.wait(tk, 100)
    assert e.value.code == gs.GS_EINVAL
    with pytest.raises(gs.GsError) as e:
        srv.poll(tk, 100)
    assert e.value.code == gs.GS_EINVAL
    srv.close()


def test_bf16_band_overflow_fails_the_request_not_the_server():
    gs, _ = _gs()
    from helpers import csr
    docs = csr([[(0, 1.0)] for _ in range(60_000)] + [[(1, 2.0)]], 4)
    idx = gs.Index.from_rows(docs, "bf16")
    srv = gs.Server(idx, max_batch=4, n_slots=1, k_max=100)
    with pytest.raises(gs.GsError) as e:
        srv.wait(srv.submit([0], [1.0], 100), 100)
    assert e.value.code == gs.GS_ECAPACITY
    ids, sc, _ = srv.wait(srv.submit([1], [1.0], 3), 3)  # the server goes on serving
    assert ids.tolist() == [60_000, 0, 1] and sc.tolist() == [2.0, 0.0, 0.0]
    assert srv.stats()["failed"] == 1
    srv.close()


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
