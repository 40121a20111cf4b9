"""Small test-only utilities: CSR construction from Python lists and random tiny instances."""
from __future__ import annotations

import numpy as np

from workload import SparseRows


def csr(rows, vocab):
    """rows: list of lists of (term, weight) -> SparseRows (term order kept as given)."""
    lens = [len(r) for r in rows]
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    terms = np.array([t for r in rows for t, _ in r], dtype=np.int32)
    weights = np.array([w for r in rows for _, w in r], dtype=np.float32)
    return SparseRows(rp, terms, weights, vocab)


def random_rows(rng, n_rows, vocab, lo, hi, weight_fn=None, sort=True):
    """Rows of distinct uniformly drawn terms; weights from weight_fn(rng, n) (default lognormal-ish)."""
    rows = []
    for _ in range(n_rows):
        n = int(rng.integers(lo, hi + 1))
        t = rng.choice(vocab, size=n, replace=False).astype(np.int32)
        if sort:
            t.sort()
        if weight_fn is None:
            w = np.log1p(rng.lognormal(0.0, 0.8, size=n)).astype(np.float32)
        else:
            w = np.asarray(weight_fn(rng, n), dtype=np.float32)
        rows.append(list(zip(t.tolist(), w.tolist())))
    return csr(rows, vocab)


def dyadic(rng, n):
    """Multiples of 1/16 in (0, 3]: every product and partial sum is exact in fp32 and fp64."""
    return rng.integers(1, 49, size=n) / 16.0


def dense(rows: SparseRows, dtype=np.float64, transform=None):
    """Dense [n_rows, vocab] matrix of a CSR (optionally mapping weights first)."""
    m = np.zeros((rows.n_rows, rows.vocab), dtype=dtype)
    w = rows.weights if transform is None else transform(rows.weights)
    for i in range(rows.n_rows):
        a, b = int(rows.row_ptr[i]), int(rows.row_ptr[i + 1])
        m[i, rows.terms[a:b]] = w[a:b]
    return m


def rank_by_score(scores, k):
    """Full sort of all docs by (score desc, id asc) via numpy.lexsort; first min(k, N) ids."""
    n = scores.shape[0]
    order = np.lexsort((np.arange(n), -scores))
    return order[: min(k, n)]


def dense_terms(docs):
    """uint8 [vocab]: 1 for terms whose doc-sorted list has every 64-posting block spanning at most 256 docs."""
    doc_of = np.repeat(np.arange(docs.n_rows), np.diff(docs.row_ptr))
    order = np.lexsort((doc_of, docs.terms))
    t_sorted, d_sorted = docs.terms[order], doc_of[order]
    starts = np.flatnonzero(np.r_[True, t_sorted[1:] != t_sorted[:-1]])
    ends = np.r_[starts[1:], len(t_sorted)]
    out = np.zeros(docs.vocab, dtype=np.uint8)
    for a, b in zip(starts, ends):
        ids = d_sorted[a:b]
        first = ids[0::64]
        last = ids[np.minimum(np.arange(0, b - a, 64) + 63, b - a - 1)]
        out[t_sorted[a]] = int(np.all(last - first <= 255))
    return out


def mixed_density_collection(rng, n_docs=53_251, vocab=320):
    # term 0: every doc; 1: every 3rd; 2: every 4th (blocks span 252 docs): byte form.
    # 3: every 5th; 4: every doc but a 300-doc hole; 5: every 2nd doc, then every 7th: 2-byte form.
    # 6: ten docs around the 8192 boundary (one block across two tiles, byte form);
    # 7: two clusters far apart in one block (2-byte form); 10.. : sparse random terms.
    d = np.arange(n_docs)
    members = {0: d, 1: d[d % 3 == 0], 2: d[d % 4 == 1], 3: d[d % 5 == 2],
               4: d[(d < 20_000) | (d >= 20_300)], 5: np.r_[d[(d < 30_000) & (d % 2 == 0)], d[(d >= 30_000) & (d % 7 == 0)]],
               6: np.arange(8190, 8200), 7: np.r_[np.arange(16_380, 16_390), np.arange(40_000, 40_003)]}
    rows = [[] for _ in range(n_docs)]
    for t, ds in members.items():
        for x in ds:
            rows[x].append(t)
    for x in range(n_docs):
        extra = rng.choice(np.arange(10, vocab), size=int(rng.integers(0, 6)), replace=False)
        rows[x].extend(int(e) for e in extra)
    out = []
    for r in rows:
        w = dyadic(rng, len(r))
        out.append(sorted(zip(r, w.tolist())))
    return csr(out, vocab)
