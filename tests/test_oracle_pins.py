"""Pins of the CPU oracle to things other than itself (CPU only).

Each test ties the oracle to a value fixed by the paper's definition and by
mathematics: a hand-worked example, dense matrix products computed by numpy,
closed forms, invariants of the inner product, and numpy's lexsort as the
brute-force ranking. A dropped term, a wrong index, a transposed operand, a
wrong sign or a wrong tie-break each fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from helpers import csr, dense, dyadic, random_rows, rank_by_score

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _queries(rows, vocab):
    return csr(rows, vocab)


# ----------------------------------------------------------- worked example --

def test_hand_worked_example_f64_and_i64():
    g = json.load(open(os.path.join(GOLDEN, "tiny_example.json")))
    docs = csr(g["docs"], g["vocab"])
    qs = _queries(g["queries"], g["vocab"])
    ids, sc = oracle.topk_f64(docs, qs, g["k"])
    assert ids.tolist() == g["expected_f64"]["ids"]
    assert sc.tolist() == g["expected_f64"]["scores"]
    ids8, sc8 = oracle.topk_i64(docs, qs, g["k"])
    assert ids8.tolist() == g["expected_i64"]["ids"]
    assert sc8.tolist() == g["expected_i64"]["scores"]
    kb = g["k_beyond_n"]
    one = _queries([g["queries"][kb["query"]]], g["vocab"])
    ids, sc = oracle.topk_f64(docs, one, [kb["k"]])
    assert ids[0].tolist() == kb["ids"]
    assert sc[0].tolist() == kb["scores"]


def test_q8_golden_values():
    ws, exp = [], []
    for line in open(os.path.join(GOLDEN, "q8_values.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        w, q = line.split()
        ws.append(float(w))
        exp.append(int(q))
    ws = np.asarray(ws, dtype=np.float32)
    assert np.all(ws.astype(np.float64) == np.asarray(ws, dtype=np.float64))
    assert oracle.q8(ws).tolist() == exp


def test_q8_matches_half_even_rounding_on_a_grid():
    # every multiple of 1/1024 in [0, 3.5]: w*85 is exact in fp64 and numpy's rint is round-half-even
    w = (np.arange(0, 3585) / 1024.0).astype(np.float32)
    expect = np.clip(np.rint(w.astype(np.float64) * 85.0), 0, 255).astype(np.uint8)
    assert np.array_equal(oracle.q8(w), expect)


# ------------------------------------------------------ dense matrix products --

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_scores_equal_dense_matmul_fp64(seed):
    rng = np.random.default_rng(seed)
    V = 512
    docs = random_rows(rng, 300, V, 1, 60)
    qs = random_rows(rng, 8, V, 0, 40, sort=False)
    S = dense(qs) @ dense(docs).T  # numpy fp64 product over the dense vocabulary
    for i in range(qs.n_rows):
        t, w = qs.row(i)
        got = oracle.scores_f64(docs, t, w)
        nz = S[i] != 0
        assert np.all(got[~nz] == 0.0)
        assert np.max(np.abs(got[nz] - S[i][nz]) / S[i][nz], initial=0.0) < 1e-13


@pytest.mark.parametrize("seed", [3, 4])
def test_topk_equals_lexsort_of_exact_dense_scores(seed):
    # dyadic weights: every sum is exact in fp64 in any order, so the ranking is fully determined
    rng = np.random.default_rng(seed)
    V = 64  # small vocabulary -> many exact ties, the tie-break rule is exercised
    docs = random_rows(rng, 400, V, 1, 12, weight_fn=dyadic)
    qs = random_rows(rng, 6, V, 1, 10, weight_fn=dyadic)
    S = dense(qs) @ dense(docs).T
    k = [1, 10, 57, 399, 400, 450]
    ids, sc = oracle.topk_f64(docs, qs, k)
    for i in range(qs.n_rows):
        exp = rank_by_score(S[i], k[i])
        assert ids[i, : len(exp)].tolist() == exp.tolist()
        assert np.array_equal(sc[i, : len(exp)], S[i][exp])
        assert np.all(ids[i, len(exp):] == -1) and np.all(sc[i, len(exp):] == 0)


@pytest.mark.parametrize("seed", [5, 6])
def test_integer_form_equals_int64_dense_matmul(seed):
    rng = np.random.default_rng(seed)
    V = 128
    docs = random_rows(rng, 500, V, 1, 30)
    qs = random_rows(rng, 6, V, 1, 25, sort=False)

    def quant(w):  # the quantiser restated with numpy's half-even rint
        return np.clip(np.rint(w.astype(np.float64) * 255.0 / 3.0), 0, 255).astype(np.int64)

    S8 = dense(qs, np.int64, quant) @ dense(docs, np.int64, quant).T
    ids, sc = oracle.topk_i64(docs, qs, 100)
    for i in range(qs.n_rows):
        t, w = qs.row(i)
        assert np.array_equal(oracle.scores_i64(docs, t, w), S8[i])
        exp = rank_by_score(S8[i], 100)
        assert ids[i].tolist() == exp.tolist()
        assert np.array_equal(sc[i], S8[i][exp])


def test_tiny_workload_against_dense_product_on_query_columns():
    w = workload.WORKLOADS["tiny-10k"]
    docs = workload.make_collection(w)
    qs = workload.make_queries(w)
    cols = np.unique(qs.terms)
    pos = {int(c): j for j, c in enumerate(cols)}
    D = np.zeros((docs.n_rows, cols.shape[0]))
    for d in range(docs.n_rows):
        t, x = docs.row(d)
        for tt, xx in zip(t, x):
            if int(tt) in pos:
                D[d, pos[int(tt)]] = xx
    Q = np.zeros((qs.n_rows, cols.shape[0]))
    for i in range(qs.n_rows):
        t, x = qs.row(i)
        Q[i, [pos[int(tt)] for tt in t]] = x
    S = Q @ D.T
    ids, sc = oracle.topk_f64(docs, qs, 100)
    for i in range(qs.n_rows):
        t, x = qs.row(i)
        got = oracle.scores_f64(docs, t, x)
        assert np.allclose(got, S[i], rtol=1e-13, atol=0)
        # the ranking agrees wherever the dense product separates neighbours by more than rounding
        exp = rank_by_score(S[i], 100)
        gap_ok = np.abs(np.diff(S[i][exp])) > 1e-12 * S[i][exp][0]
        same = ids[i] == exp
        assert np.all(same[:-1][gap_ok] | ~gap_ok)
        assert np.allclose(sc[i], S[i][ids[i]], rtol=1e-13, atol=0)


# ------------------------------------------------------------- closed forms --

def test_single_term_query_closed_form():
    rng = np.random.default_rng(7)
    V = 40
    docs = random_rows(rng, 300, V, 1, 8)
    t = 5
    wq = np.float32(1.25)
    qs = _queries([[(t, float(wq))]], V)
    holders, wd = [], []
    for d in range(docs.n_rows):
        tt, ww = docs.row(d)
        hit = np.nonzero(tt == t)[0]
        if hit.size:
            holders.append(d)
            wd.append(float(ww[hit[0]]))
    # expected: t's posting list by (w_d desc, id asc), then the other docs by id
    order = sorted(range(len(holders)), key=lambda j: (-wd[j], holders[j]))
    rest = [d for d in range(docs.n_rows) if d not in set(holders)]
    exp_ids = [holders[j] for j in order] + rest
    exp_sc = [float(wq) * wd[j] for j in order] + [0.0] * len(rest)
    ids, sc = oracle.topk_f64(docs, qs, [docs.n_rows])
    assert ids[0].tolist() == exp_ids
    assert sc[0].tolist() == exp_sc


def test_all_ones_weights_count_shared_terms():
    rng = np.random.default_rng(8)
    V = 50
    docs = random_rows(rng, 200, V, 1, 20, weight_fn=lambda r, n: np.ones(n))
    qs = random_rows(rng, 5, V, 1, 15, weight_fn=lambda r, n: np.ones(n))
    for i in range(qs.n_rows):
        qt = set(qs.row(i)[0].tolist())
        expect = np.array([len(qt & set(docs.row(d)[0].tolist())) for d in range(docs.n_rows)], dtype=np.float64)
        t, w = qs.row(i)
        assert np.array_equal(oracle.scores_f64(docs, t, w), expect)
        assert np.array_equal(oracle.scores_i64(docs, t, w), expect.astype(np.int64) * 85 * 85)


def test_empty_query_and_k_beyond_n():
    rng = np.random.default_rng(9)
    docs = random_rows(rng, 7, 30, 1, 5)
    qs = _queries([[]], 30)
    ids, sc = oracle.topk_f64(docs, qs, [10])
    assert ids[0].tolist() == [0, 1, 2, 3, 4, 5, 6, -1, -1, -1]
    assert np.all(sc == 0)
    ids, sc = oracle.topk_i64(docs, qs, [3], k_max=5)
    assert ids[0].tolist() == [0, 1, 2, -1, -1]


def test_k_zero_and_empty_collection():
    docs = csr([], 10)
    qs = _queries([[(1, 1.0)]], 10)
    ids, sc = oracle.topk_f64(docs, qs, [3])
    assert ids.tolist() == [[-1, -1, -1]]
    rng = np.random.default_rng(10)
    docs = random_rows(rng, 5, 10, 1, 3)
    ids, sc = oracle.topk_f64(docs, qs, [0], k_max=2)
    assert ids.tolist() == [[-1, -1]]


def test_invalid_queries_are_rejected():
    rng = np.random.default_rng(11)
    docs = random_rows(rng, 5, 10, 1, 3)
    with pytest.raises(ValueError):
        oracle.topk_f64(docs, _queries([[(1, 1.0), (1, 2.0)]], 10), [2])  # duplicate term
    with pytest.raises(ValueError):
        oracle.topk_f64(docs, _queries([[(10, 1.0)]], 10), [2])  # term out of range
    with pytest.raises(ValueError):
        oracle.topk_f64(docs, _queries([[(3, float("nan"))]], 10), [2])


# --------------------------------------------------------------- invariants --

def test_only_shared_terms_contribute():
    rng = np.random.default_rng(12)
    V = 200
    docs = random_rows(rng, 150, V, 1, 20)
    qs = random_rows(rng, 4, V, 1, 20)
    qterms = set(qs.terms.tolist())
    free = np.array(sorted(set(range(V)) - qterms), dtype=np.int32)
    # add non-query terms with arbitrary weights to every doc
    rows = []
    for d in range(docs.n_rows):
        t, w = docs.row(d)
        extra = rng.choice(free[~np.isin(free, t)], size=5, replace=False)
        r = list(zip(t.tolist(), w.tolist())) + [(int(e), float(rng.uniform(0.1, 3.0))) for e in extra]
        r.sort()
        rows.append(r)
    docs2 = csr(rows, V)
    for i in range(qs.n_rows):
        t, w = qs.row(i)
        assert np.array_equal(oracle.scores_f64(docs, t, w), oracle.scores_f64(docs2, t, w))


def test_linearity_in_query_weights():
    rng = np.random.default_rng(13)
    V = 300
    docs = random_rows(rng, 200, V, 1, 40)
    qs = random_rows(rng, 6, V, 2, 30)
    for i in range(qs.n_rows):
        t, w = qs.row(i)
        s1 = oracle.scores_f64(docs, t, w)
        # doubling is exact in fp32 and commutes with every fp64 rounding
        assert np.array_equal(oracle.scores_f64(docs, t, w * np.float32(2)), 2.0 * s1)
        # additivity over a split of the query into two term-disjoint halves
        h = len(t) // 2
        s_a = oracle.scores_f64(docs, t[:h], w[:h])
        s_b = oracle.scores_f64(docs, t[h:], w[h:])
        nz = s1 != 0
        assert np.all((s_a + s_b)[~nz] == 0)
        assert np.max(np.abs(s_a + s_b - s1)[nz] / s1[nz], initial=0) < 1e-13


def test_doc_permutation_equivariance():
    rng = np.random.default_rng(14)
    V = 100
    docs = random_rows(rng, 250, V, 1, 15)
    qs = random_rows(rng, 4, V, 1, 12)
    perm = rng.permutation(docs.n_rows)  # new doc j is old doc perm[j]
    docs_p = docs.subset(perm)
    k = [250] * qs.n_rows
    ids, sc = oracle.topk_f64(docs, qs, k)
    ids_p, sc_p = oracle.topk_f64(docs_p, qs, k)
    for i in range(qs.n_rows):
        assert np.array_equal(sc[i], sc_p[i])
        mapped = perm[ids_p[i]]
        # ids agree through the permutation except inside runs of exactly equal scores
        for s in np.unique(sc[i]):
            a = set(ids[i][sc[i] == s].tolist())
            b = set(mapped[sc_p[i] == s].tolist())
            assert a == b


def test_unsorted_document_rows_give_the_same_scores():
    rng = np.random.default_rng(15)
    V = 80
    docs = random_rows(rng, 100, V, 2, 20)
    rows = []
    for d in range(docs.n_rows):
        t, w = docs.row(d)
        p = rng.permutation(len(t))
        rows.append(list(zip(t[p].tolist(), w[p].tolist())))
    docs_u = csr(rows, V)
    qs = random_rows(rng, 3, V, 1, 20)
    for i in range(qs.n_rows):
        t, w = qs.row(i)
        assert np.array_equal(oracle.scores_f64(docs, t, w), oracle.scores_f64(docs_u, t, w))


def test_pair_scores_match_dense_vector():
    w = workload.WORKLOADS["tiny-10k"]
    docs = workload.make_collection(w)
    qs = workload.make_queries(w)
    t, x = qs.row(3)
    full = oracle.scores_f64(docs, t, x)
    fulli = oracle.scores_i64(docs, t, x)
    pick = np.array([0, 17, 4096, 9999], dtype=np.int32)
    f, i = oracle.pair_scores(docs, t, x, pick)
    assert np.array_equal(f, full[pick])
    assert np.array_equal(i, fulli[pick])
