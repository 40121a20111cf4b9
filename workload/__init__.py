"""Seeded synthetic workloads shaped like the paper's MS MARCO + SPLADE data.

This module synthesises inputs only. It holds none of the retrieval method's
arithmetic, and it is the one piece shared by the CPU oracle (``oracle/``) and
the GPU library (``paper_2606_26441_amd``). The row sampler is C
(``workload/gen.c``) so that the 8.8M-passage collection (about 1.06 B postings)
is synthesised in seconds, deterministically and independently of the number of
threads.

The paper's statistics (Sec. 6.1 "Data"): 8.8M passages, 30,522-term
vocabulary, ~127 terms per passage, ~50 per query, weights log(1+ReLU(.)) in
[0, 3.5]. The stand-in laws used here:

* doc nnz ~ Poisson(120) clipped to [8, 400];
* distinct term ids per row: Zipf(s=1.1) over ranks 1..30,522 sampled without
  replacement, ranks mapped through a seeded vocabulary permutation;
* weight = float32(log1p(lognormal(0, 0.8))) capped at 3.0;
* queries: nnz ~ Poisson(30) clipped to [1, 250] (plain batches) or
  round(lognormal(median 25, sigma 0.8)) clipped to [5, 250] (long-tailed
  batches), same term and weight laws.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgswl.so")
_lib = None

VOCAB = 30522
ZIPF_S = 1.1
W_SIGMA = 0.8
W_CAP = 3.0
PERM_SEED = 0

KIND_DOCS = 1
KIND_QUERIES = 2

LAW_POISSON = 0
LAW_LOGNORMAL = 1


def build(force: bool = True) -> str:
    """Compile the row sampler with gcc (OpenMP). Returns the library path."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i32, i64, u64, f64, f32, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_float, ctypes.c_void_p)
    lib.wl_row_nnz.argtypes = [u64, i32, i64, i32, f64, f64, i64, i64, i32, vp]
    lib.wl_row_nnz.restype = ctypes.c_int
    lib.wl_fill_rows.argtypes = [u64, i32, i64, i32, f64, f64, i64, i64, i32, f64, u64, f64, f32,
                                 vp, vp, vp]
    lib.wl_fill_rows.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclasses.dataclass
class SparseRows:
    """Row-major CSR: row_ptr[n+1] int64, terms[nnz] int32 (ascending per row), weights[nnz] float32."""
    row_ptr: np.ndarray
    terms: np.ndarray
    weights: np.ndarray
    vocab: int = VOCAB

    @property
    def n_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row(self, i: int):
        a, b = int(self.row_ptr[i]), int(self.row_ptr[i + 1])
        return self.terms[a:b], self.weights[a:b]

    def subset(self, rows) -> "SparseRows":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.row_ptr[rows + 1] - self.row_ptr[rows]
        rp = np.zeros(rows.shape[0] + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        idx = np.concatenate([np.arange(self.row_ptr[r], self.row_ptr[r + 1]) for r in rows]) \
            if rows.shape[0] else np.zeros(0, dtype=np.int64)
        return SparseRows(rp, self.terms[idx].copy(), self.weights[idx].copy(), self.vocab)

    def digest(self) -> str:
        h = hashlib.sha256()
        for a in (self.row_ptr, self.terms, self.weights):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def sample_rows(n_rows: int, seed: int, kind: int, law: int, a: float, b: float, lo: int, hi: int,
                vocab: int = VOCAB, zipf_s: float = ZIPF_S, perm_seed: int = PERM_SEED,
                w_sigma: float = W_SIGMA, w_cap: float = W_CAP) -> SparseRows:
    lib = _load()
    nnz = np.empty(n_rows, dtype=np.int64)
    rc = lib.wl_row_nnz(seed, kind, n_rows, law, a, b, lo, hi, vocab, nnz.ctypes.data)
    if rc != 0:
        raise ValueError("wl_row_nnz failed (%d)" % rc)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(nnz, out=row_ptr[1:])
    total = int(row_ptr[-1])
    terms = np.empty(total, dtype=np.int32)
    weights = np.empty(total, dtype=np.float32)
    rc = lib.wl_fill_rows(seed, kind, n_rows, law, a, b, lo, hi, vocab, zipf_s, perm_seed, w_sigma,
                          w_cap, row_ptr.ctypes.data, terms.ctypes.data, weights.ctypes.data)
    if rc != 0:
        raise RuntimeError("wl_fill_rows failed (%d)" % rc)
    return SparseRows(row_ptr, terms, weights, vocab)


def collection(n_docs: int, seed: int = 1, mean_nnz: float = 120.0, lo: int = 8, hi: int = 400,
               vocab: int = VOCAB) -> SparseRows:
    """Doc-major collection: nnz ~ Poisson(mean) clipped to [lo, hi]."""
    return sample_rows(n_docs, seed, KIND_DOCS, LAW_POISSON, mean_nnz, 0.0, lo, hi, vocab)


def queries_poisson(n: int, seed: int = 2, mean_nnz: float = 30.0, lo: int = 1, hi: int = 250,
                    vocab: int = VOCAB) -> SparseRows:
    return sample_rows(n, seed, KIND_QUERIES, LAW_POISSON, mean_nnz, 0.0, lo, hi, vocab)


def queries_lognormal(n: int, seed: int = 2, median: float = 25.0, sigma: float = 0.8, lo: int = 5,
                      hi: int = 250, vocab: int = VOCAB) -> SparseRows:
    return sample_rows(n, seed, KIND_QUERIES, LAW_LOGNORMAL, median, sigma, lo, hi, vocab)


def k_mix(n: int, seed: int = 4, choices=(10, 100, 1000)) -> np.ndarray:
    """Per-query k drawn uniformly from ``choices`` (long-tailed batch and serving workloads)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(np.asarray(choices, dtype=np.int32), size=n).astype(np.int32)


def poisson_arrivals(rate_qps: float, duration_s: float, seed: int = 3) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate_qps * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_qps, size=n))
    return t[t < duration_s]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_docs: int
    n_queries: int
    query_law: str  # "poisson" | "lognormal"
    ks: tuple
    doc_seed: int = 1
    query_seed: int = 2


WORKLOADS = {
    "tiny-10k": Workload("tiny-10k", 10_000, 8, "poisson", (10, 100), doc_seed=11, query_seed=12),
    "mid-1m": Workload("mid-1m", 1_000_000, 500, "poisson", (1000,), doc_seed=21, query_seed=22),
    "full-8.8m": Workload("full-8.8m", 8_800_000, 500, "poisson", (10, 1000), doc_seed=31, query_seed=32),
    "uneven-8.8m": Workload("uneven-8.8m", 8_800_000, 4096, "lognormal", (10, 100, 1000),
                            doc_seed=31, query_seed=42),
}


def make_queries(w: Workload, n: Optional[int] = None, seed: Optional[int] = None) -> SparseRows:
    n = w.n_queries if n is None else n
    seed = w.query_seed if seed is None else seed
    if w.query_law == "poisson":
        return queries_poisson(n, seed=seed)
    return queries_lognormal(n, seed=seed)


def make_collection(w: Workload, n_docs: Optional[int] = None) -> SparseRows:
    return collection(w.n_docs if n_docs is None else n_docs, seed=w.doc_seed)
