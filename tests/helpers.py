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
