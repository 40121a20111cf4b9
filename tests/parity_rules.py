"""Acceptance rules that compare a GPU top-k result with the CPU oracle (test code).

* fp32: every returned score is within REL_TOL of the exact fp64 score of its
  document (exactly 0 when that score is 0); the list is non-increasing, ties in
  the returned scores are ordered by ascending doc id; a returned id outside the
  oracle's top-k scores at least s_k*(1-REL_TOL) and an oracle id missing from
  the result scores at most s_k*(1+REL_TOL), where s_k is the oracle's k-th
  score (swaps are allowed only inside the tolerance band of the k-th score).
* uint8 impacts: ids and int32 scores bit-exact against the integer oracle.
* bf16 with fp64 boundary rescoring: ids identical to the fp64 oracle and scores
  bitwise equal to the oracle's fp64 values.
"""
from __future__ import annotations

import numpy as np

import oracle

REL_TOL = 1e-5


def check_fp32(docs, q_terms, q_weights, ids, scores, ref_ids, ref_scores, k, tol=REL_TOL, what=""):
    n = docs.n_rows
    kq = min(int(k), n)
    ids = np.asarray(ids)
    scores = np.asarray(scores, dtype=np.float64)
    assert np.all(ids[kq:] == -1) and np.all(scores[kq:] == 0), what + ": padding"
    ids, scores = ids[:kq], scores[:kq]
    assert np.all((ids >= 0) & (ids < n)), what + ": id range"
    assert np.unique(ids).shape[0] == kq, what + ": duplicate ids"
    exact, _ = oracle.pair_scores(docs, q_terms, q_weights, ids)
    zero = exact == 0
    assert np.all(scores[zero] == 0), what + ": score of a non-matching doc"
    rel = np.abs(scores[~zero] - exact[~zero]) / exact[~zero]
    assert rel.size == 0 or rel.max() <= tol, what + ": score error %.3g" % rel.max()
    assert np.all(np.diff(scores) <= 0), what + ": not sorted"
    same = np.diff(scores) == 0
    assert np.all(np.diff(ids)[same] > 0), what + ": tie order"
    if kq == 0:
        return
    s_k = float(ref_scores[kq - 1])
    ref = set(np.asarray(ref_ids[:kq]).tolist())
    got = set(ids.tolist())
    extra = np.array(sorted(got - ref), dtype=np.int32)
    if extra.size:
        e, _ = oracle.pair_scores(docs, q_terms, q_weights, extra)
        assert np.all(e >= s_k * (1 - tol)), what + ": id outside the tolerance band"
    missing = np.array(sorted(ref - got), dtype=np.int32)
    if missing.size:
        m, _ = oracle.pair_scores(docs, q_terms, q_weights, missing)
        assert np.all(m <= s_k * (1 + tol)), what + ": oracle id missing outside the tolerance band"


def check_exact_int(ids, scores, ref_ids, ref_scores, what=""):
    assert np.array_equal(np.asarray(ids), np.asarray(ref_ids)), what + ": ids differ"
    assert np.array_equal(np.asarray(scores).astype(np.int64), np.asarray(ref_scores)), what + ": scores differ"


def check_exact_f64(ids, scores, ref_ids, ref_scores, what=""):
    assert np.array_equal(np.asarray(ids), np.asarray(ref_ids)), what + ": ids differ"
    a = np.asarray(scores, dtype=np.float64)
    b = np.asarray(ref_scores, dtype=np.float64)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), what + ": scores differ"


def check_batch(precision, docs, queries, ids, scores, k, n_threads=0, what=""):
    """Full oracle comparison for every query of a batch."""
    k = np.broadcast_to(np.asarray(k, dtype=np.int32), (queries.n_rows,))
    k_max = ids.shape[1]
    if precision == "u8":
        rid, rsc = oracle.topk_i64(docs, queries, k, k_max=k_max, n_threads=n_threads)
        for q in range(queries.n_rows):
            check_exact_int(ids[q], scores[q], rid[q], rsc[q], "%s q%d" % (what, q))
        return
    rid, rsc = oracle.topk_f64(docs, queries, k, k_max=k_max, n_threads=n_threads)
    for q in range(queries.n_rows):
        if precision == "bf16":
            check_exact_f64(ids[q], scores[q], rid[q], rsc[q], "%s q%d" % (what, q))
        else:
            t, w = queries.row(q)
            check_fp32(docs, t, w, ids[q], scores[q], rid[q], rsc[q], k[q], what="%s q%d" % (what, q))
