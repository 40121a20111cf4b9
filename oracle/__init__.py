"""CPU oracle for exact learned-sparse retrieval (fp64 and int64).

TEST INFRASTRUCTURE: only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg import this package. The GPU library never does,
and the two share no code (see ``oracle/oracle.c`` for what is computed and
which passages of the paper it follows).

Every function here is a thin ctypes wrapper over ``oracle.c``:

* ``topk_f64`` - exact top-k of S(q,d) = sum over shared terms of
  w_q(t) * w_d(t) in fp64, full sort by (score desc, doc id asc);
* ``topk_i64`` - the same on uint8 impacts q8(w) = round(w*255/3) (ties to
  even, saturated at 255) with exact int64 sums;
* ``scores_f64`` / ``scores_i64`` - the dense score vector of one query;
* ``pair_scores`` - S(q,d) for a list of documents (sampled checks at full
  scale);
* ``q8`` - the quantiser.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over queries)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", _SRC, "-o", tmp,
           "-lm"]
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
    i32, i64, vp, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_float
    lib.oracle_q8.argtypes = [f32]
    lib.oracle_q8.restype = ctypes.c_uint8
    lib.oracle_q8_array.argtypes = [vp, i64, vp]
    lib.oracle_q8_array.restype = None
    for name in ("oracle_scores_f64", "oracle_scores_i64"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, vp, i64, i32, vp, vp, i64, vp]
        fn.restype = ctypes.c_int
    lib.oracle_pair_scores.argtypes = [vp, vp, vp, i64, i32, vp, vp, i64, vp, i64, vp, vp]
    lib.oracle_pair_scores.restype = ctypes.c_int
    for name in ("oracle_topk_f64", "oracle_topk_i64"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, vp, i64, i32, vp, i32, vp, vp, vp, i32, vp, vp, i32]
        fn.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _check(rc, what):
    if rc == -1:
        raise ValueError("%s: invalid input" % what)
    if rc != 0:
        raise MemoryError("%s failed (%d)" % (what, rc))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def q8(w) -> np.ndarray:
    w = _c(w, np.float32).reshape(-1)
    out = np.empty(w.shape[0], dtype=np.uint8)
    _load().oracle_q8_array(w.ctypes.data, w.shape[0], out.ctypes.data)
    return out


def _docs(docs):
    rp, t, w = _c(docs.row_ptr, np.int64), _c(docs.terms, np.int32), _c(docs.weights, np.float32)
    return rp, t, w, rp.shape[0] - 1, int(getattr(docs, "vocab", 30522))


def scores_f64(docs, q_terms, q_weights) -> np.ndarray:
    rp, t, w, n, V = _docs(docs)
    qt, qw = _c(q_terms, np.int32), _c(q_weights, np.float32)
    out = np.empty(n, dtype=np.float64)
    _check(_load().oracle_scores_f64(rp.ctypes.data, t.ctypes.data, w.ctypes.data, n, V, qt.ctypes.data,
                                     qw.ctypes.data, qt.shape[0], out.ctypes.data), "scores_f64")
    return out


def scores_i64(docs, q_terms, q_weights) -> np.ndarray:
    rp, t, w, n, V = _docs(docs)
    qt, qw = _c(q_terms, np.int32), _c(q_weights, np.float32)
    out = np.empty(n, dtype=np.int64)
    _check(_load().oracle_scores_i64(rp.ctypes.data, t.ctypes.data, w.ctypes.data, n, V, qt.ctypes.data,
                                     qw.ctypes.data, qt.shape[0], out.ctypes.data), "scores_i64")
    return out


def pair_scores(docs, q_terms, q_weights, doc_ids):
    """(fp64 scores, int64 scores) of one query against the listed documents."""
    rp, t, w, n, V = _docs(docs)
    qt, qw = _c(q_terms, np.int32), _c(q_weights, np.float32)
    ids = _c(doc_ids, np.int32).reshape(-1)
    f = np.empty(ids.shape[0], dtype=np.float64)
    i = np.empty(ids.shape[0], dtype=np.int64)
    _check(_load().oracle_pair_scores(rp.ctypes.data, t.ctypes.data, w.ctypes.data, n, V, qt.ctypes.data,
                                      qw.ctypes.data, qt.shape[0], ids.ctypes.data, ids.shape[0],
                                      f.ctypes.data, i.ctypes.data), "pair_scores")
    return f, i


def _topk(name, score_dtype, docs, queries, k, k_max=None, n_threads=0):
    rp, t, w, n, V = _docs(docs)
    qrp, qt, qw = _c(queries.row_ptr, np.int64), _c(queries.terms, np.int32), _c(queries.weights, np.float32)
    nq = qrp.shape[0] - 1
    k = np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)).copy()
    k_max = int(k.max()) if (k_max is None and nq) else int(k_max or 0)
    ids = np.empty((nq, k_max), dtype=np.int32)
    sc = np.empty((nq, k_max), dtype=score_dtype)
    _check(getattr(_load(), name)(rp.ctypes.data, t.ctypes.data, w.ctypes.data, n, V, qrp.ctypes.data, nq,
                                  qt.ctypes.data, qw.ctypes.data, k.ctypes.data, k_max, ids.ctypes.data,
                                  sc.ctypes.data, int(n_threads)), name)
    return ids, sc


def topk_f64(docs, queries, k, k_max=None, n_threads=0):
    """Exact fp64 top-k: (ids [nq, k_max] int32, scores [nq, k_max] float64)."""
    return _topk("oracle_topk_f64", np.float64, docs, queries, k, k_max, n_threads)


def topk_i64(docs, queries, k, k_max=None, n_threads=0):
    """Exact uint8-impact top-k: (ids [nq, k_max] int32, scores [nq, k_max] int64)."""
    return _topk("oracle_topk_i64", np.int64, docs, queries, k, k_max, n_threads)
