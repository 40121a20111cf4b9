"""Host posting layout built by the library (same code as the device index build), checked on CPU."""
import numpy as np
import pytest

import oracle
import workload
from helpers import random_rows


def _bf16_rne(w):
    u = np.asarray(w, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


@pytest.fixture(scope="module")
def small():
    return workload.collection(3000, seed=77)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "u8"])
def test_layout_properties(small, precision):
    import paper_2606_26441_amd as gs
    L = gs.layout_host(small.row_ptr, small.terms, small.weights, small.vocab, precision)
    V = small.vocab
    off, ln, doc, w = L["term_off"], L["term_len"], L["post_doc"], L["post_w"]
    df = np.bincount(small.terms, minlength=V)
    assert np.array_equal(ln, df)
    assert off[0] == 0 and np.all(np.diff(off) == (df + 63) // 64 * 64)
    assert off[-1] == doc.shape[0] and doc.shape[0] % 64 == 0
    # expected (doc, weight) per term from the doc-major input
    doc_of = np.repeat(np.arange(small.n_rows), np.diff(small.row_ptr))
    order = np.lexsort((doc_of, small.terms))
    exp_w = small.weights[order]
    if precision == "bf16":
        exp_w = _bf16_rne(exp_w)
    elif precision == "u8":
        exp_w = oracle.q8(exp_w).astype(np.float32)
    pos = np.concatenate([np.arange(off[t], off[t] + df[t]) for t in range(V) if df[t]])
    assert np.array_equal(doc[pos], doc_of[order])  # every posting once, doc-sorted within its term
    assert np.array_equal(w[pos], exp_w)
    pad = np.ones(doc.shape[0], bool)
    pad[pos] = False
    assert np.all(doc[pad] == -1) and np.all(w[pad] == 0)
    nb = doc.shape[0] // 64
    assert np.array_equal(L["blk_max"], w.reshape(nb, 64).max(axis=1))
    assert np.array_equal(L["blk_first_doc"], doc.reshape(nb, 64)[:, 0])


def test_unsorted_rows_give_the_same_layout():
    import paper_2606_26441_amd as gs
    rng = np.random.default_rng(3)
    rows = random_rows(rng, 200, 50, 1, 20, sort=True)
    L1 = gs.layout_host(rows.row_ptr, rows.terms, rows.weights, 50)
    t2, w2 = rows.terms.copy(), rows.weights.copy()
    for i in range(rows.n_rows):
        a, b = rows.row_ptr[i], rows.row_ptr[i + 1]
        p = rng.permutation(b - a) + a
        t2[a:b], w2[a:b] = rows.terms[p], rows.weights[p]
    L2 = gs.layout_host(rows.row_ptr, t2, w2, 50)
    for k in L1:
        assert np.array_equal(L1[k], L2[k])


def test_empty_rows_and_unused_terms():
    import paper_2606_26441_amd as gs
    rp = np.array([0, 0, 2, 2, 3], np.int64)
    t = np.array([3, 5, 3], np.int32)
    w = np.array([1.0, 2.0, 0.25], np.float32)
    L = gs.layout_host(rp, t, w, 8)
    assert L["term_len"].tolist() == [0, 0, 0, 2, 0, 1, 0, 0]
    assert L["term_off"].tolist() == [0, 0, 0, 0, 64, 64, 128, 128, 128]
    assert L["post_doc"][:3].tolist() == [1, 3, -1] and L["post_doc"][64] == 1


def test_byte_form_of_dense_terms():
    # The byte form must rebuild every doc id of a dense term from its block's first doc, and
    # the dense flags must match a classification done here from the rows themselves.
    import paper_2606_26441_amd as gs
    from helpers import dense_terms, mixed_density_collection
    docs = mixed_density_collection(np.random.default_rng(77))
    L = gs.layout_host(docs.row_ptr, docs.terms, docs.weights, docs.vocab, "fp32")
    expect = dense_terms(docs)
    assert list(np.flatnonzero(expect)) == [0, 1, 2, 6]
    assert np.array_equal(L["term_dense"], expect)
    P = L["post_doc"].shape[0]
    real = np.zeros(P, dtype=bool)
    in_dense = np.zeros(P, dtype=bool)
    for v in range(docs.vocab):
        a, n = int(L["term_off"][v]), int(L["term_len"][v])
        real[a:a + n] = True
        in_dense[a:a + n] = bool(expect[v])
    base = np.repeat(L["blk_first_doc"], 64)
    rebuilt = base[in_dense] + L["post_b8"][in_dense].astype(np.int64)
    assert np.array_equal(rebuilt, L["post_doc"][in_dense])
    assert not L["post_b8"][~in_dense].any()
    # the flagged terms are exactly those whose blocks stay within 256 docs
    for v in np.flatnonzero(expect):
        a, n = int(L["term_off"][v]), int(L["term_len"][v])
        d = L["post_doc"][a:a + n]
        spans = [d[k:k + 64][-1] - d[k] for k in range(0, n, 64)]
        assert max(spans) <= 255
