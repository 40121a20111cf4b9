"""Python binding of libgpusparse.so: exact learned-sparse retrieval on MI355X.

Argument marshalling only. Every step of index build and search runs in the
C++/HIP library behind ``include/gpusparse.h``; PyTorch provides device memory
(workspace and output tensors) and the HIP stream. Importing this module fails
when the library has not been built (``python paper_2606_26441_amd/build.py``):
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

import torch  # loads the HIP runtime that the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpusparse.so")

GS_OK, GS_EINVAL, GS_ENOMEM, GS_EHIP, GS_ECAPACITY, GS_EUNSUPPORTED, GS_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
GS_FP32, GS_BF16, GS_U8 = 0, 1, 2
GS_KEEP_FORWARD, GS_KEEP_DOC_IDS = 1, 2
GS_KERNEL_AUTO, GS_KERNEL_TILED, GS_KERNEL_ATOMIC, GS_KERNEL_DOCPAR, GS_KERNEL_SHARED, GS_KERNEL_GROUP = 0, 1, 2, 3, 4, 5
GS_MAX_K = 4096
GS_MAX_QUERY_NNZ = 256

PRECISIONS = {"fp32": GS_FP32, "bf16": GS_BF16, "u8": GS_U8}
KERNELS = {"auto": GS_KERNEL_AUTO, "tiled": GS_KERNEL_TILED, "atomic": GS_KERNEL_ATOMIC,
           "docpar": GS_KERNEL_DOCPAR, "shared": GS_KERNEL_SHARED, "group": GS_KERNEL_GROUP}
SCORE_DTYPES = {GS_FP32: torch.float32, GS_BF16: torch.float64, GS_U8: torch.int32}


class GsError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed: %s (%d): %s" % (where, _STATUS.get(code, "?"), code, msg))
        self.code = code


_STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "HIP error", -4: "capacity exceeded",
           -5: "unsupported", -6: "timeout"}


class SearchOpts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("query_tile", ctypes.c_int32), ("tile_docs", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("no_fused_filter", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("memory_budget", ctypes.c_int64), ("search", SearchOpts)]


class ServerStats(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("device_steps", ctypes.c_int64), ("mean_batch", ctypes.c_double),
                ("max_in_flight", ctypes.c_int64), ("pending", ctypes.c_int64), ("arena_rows", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("row_bytes", ctypes.c_int64)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n_docs", ctypes.c_int64), ("nnz", ctypes.c_int64), ("padded_nnz", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("vocab_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tile_grain", ctypes.c_int32), ("n_tiles", ctypes.c_int64),
                ("n_dense_terms", ctypes.c_int64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgpusparse.so is not built (run: python paper_2606_26441_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    lib.gs_version.restype = ctypes.c_char_p
    lib.gs_status_string.argtypes = [i32]
    lib.gs_status_string.restype = ctypes.c_char_p
    lib.gs_last_error.restype = ctypes.c_char_p
    lib.gs_debug_fail_alloc.argtypes = [i64]
    lib.gs_debug_fail_alloc.restype = i32
    lib.gs_build_index.argtypes = [vp, i64, vp, vp, i64, i32, i32, u32, vp, P(vp)]
    lib.gs_build_index.restype = i32
    lib.gs_index_info.argtypes = [vp, P(IndexInfo)]
    lib.gs_index_info.restype = i32
    lib.gs_index_dense_terms.argtypes = [vp, vp, i32]
    lib.gs_index_dense_terms.restype = i32
    lib.gs_free_index.argtypes = [vp]
    lib.gs_free_index.restype = None
    lib.gs_layout_host.argtypes = [vp, i64, vp, vp, i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.gs_layout_host.restype = i32
    lib.gs_query_plan_host.argtypes = [i32, vp, vp, vp, i32, P(i32), P(ctypes.c_double), P(ctypes.c_double)]
    lib.gs_query_plan_host.restype = i32
    lib.gs_batch_create.argtypes = [vp, vp, i32, vp, vp, i64, vp, i32, vp, P(vp)]
    lib.gs_batch_create.restype = i32
    lib.gs_batch_free.argtypes = [vp]
    lib.gs_batch_free.restype = None
    lib.gs_batch_reserve.argtypes = [vp, i32, i64, i32, P(vp)]
    lib.gs_batch_reserve.restype = i32
    lib.gs_batch_update.argtypes = [vp, vp, i32, vp, vp, i64, vp, vp]
    lib.gs_batch_update.restype = i32
    lib.gs_graph_create.argtypes = [vp, vp, vp, sz, vp, vp, P(SearchOpts), vp, P(vp)]
    lib.gs_graph_create.restype = i32
    lib.gs_graph_launch.argtypes = [vp, vp]
    lib.gs_graph_launch.restype = i32
    lib.gs_graph_free.argtypes = [vp]
    lib.gs_graph_free.restype = None
    lib.gs_autotune.argtypes = [vp, vp, vp, sz, vp, vp, i32, vp, P(SearchOpts), vp, vp, i32, P(i32)]
    lib.gs_autotune.restype = i32
    lib.gs_server_create.argtypes = [vp, P(ServerOpts), P(vp)]
    lib.gs_server_create.restype = i32
    lib.gs_server_submit.argtypes = [vp, vp, vp, i32, i32]
    lib.gs_server_submit.restype = i64
    lib.gs_server_wait.argtypes = [vp, i64, i32, vp, vp, P(ctypes.c_double)]
    lib.gs_server_wait.restype = i32
    lib.gs_server_poll.argtypes = [vp, i64, vp, vp, P(ctypes.c_double)]
    lib.gs_server_poll.restype = i32
    lib.gs_server_stats.argtypes = [vp, P(ServerStats)]
    lib.gs_server_stats.restype = i32
    lib.gs_server_destroy.argtypes = [vp]
    lib.gs_server_destroy.restype = None
    lib.gs_search_workspace_size.argtypes = [vp, i32, i64, i32, P(SearchOpts), P(sz)]
    lib.gs_search_workspace_size.restype = i32
    lib.gs_workspace_size.argtypes = [vp, i32, P(SearchOpts), P(sz)]
    lib.gs_workspace_size.restype = i32
    lib.gs_search_batch.argtypes = [vp, vp, vp, sz, vp, vp, P(SearchOpts), vp]
    lib.gs_search_batch.restype = i32
    lib.gs_search_batch_noalloc.argtypes = [vp, vp, vp, vp, P(SearchOpts), vp]
    lib.gs_search_batch_noalloc.restype = i32
    lib.gs_search.argtypes = [vp, vp, i32, vp, vp, i64, vp, i32, vp, sz, vp, vp, P(SearchOpts), vp]
    lib.gs_search.restype = i32
    lib.gs_batch_diagnostics.argtypes = [vp, vp]
    lib.gs_batch_diagnostics.restype = i32
    lib.gs_device_copy.argtypes = [vp, vp, sz, vp]
    lib.gs_device_copy.restype = i32
    lib.gs_lds_atomic_probe.argtypes = [i32, i32, i32, i32, vp, vp, P(i64)]
    lib.gs_lds_atomic_probe.restype = i32
    lib.gs_timing_enable.argtypes = [i32]
    lib.gs_timing_enable.restype = i32
    lib.gs_timing_read.argtypes = [P(ctypes.c_double), P(i64), P(ctypes.c_double), P(i64)]
    lib.gs_timing_read.restype = i32
    return lib


lib = _load()


def _check(rc: int, where: str):
    if rc != GS_OK:
        raise GsError(rc, where, lib.gs_last_error().decode())


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _stream_ptr(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def make_opts(kernel="auto", query_tile=0, tile_docs=0, chunk=0, fused_filter=True, prune=False) -> SearchOpts:
    o = SearchOpts()
    o.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.query_tile, o.tile_docs, o.chunk = int(query_tile), int(tile_docs), int(chunk)
    o.no_fused_filter = 0 if fused_filter else 1
    o.prune = 1 if prune else 0
    return o


def layout_host(row_ptr, terms, weights, vocab: int, precision="fp32"):
    """Host-only posting layout (same code as the device index build), as numpy arrays."""
    rp, t, w = _np(row_ptr, np.int64), _np(terms, np.int32), _np(weights, np.float32)
    n = rp.shape[0] - 1
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    padded = ctypes.c_int64(0)
    _check(lib.gs_layout_host(rp.ctypes.data, n, t.ctypes.data, w.ctypes.data, t.shape[0], vocab, prec,
                              ctypes.addressof(padded), None, None, None, None, None, None, None, None),
           "gs_layout_host")
    P = padded.value
    out = dict(term_off=np.empty(vocab + 1, np.int64), term_len=np.empty(vocab, np.int32),
               post_doc=np.empty(P, np.int32), post_w=np.empty(P, np.float32),
               blk_max=np.empty(P // 64, np.float32), blk_first_doc=np.empty(P // 64, np.int32),
               term_dense=np.empty(vocab, np.uint8), post_b8=np.empty(P, np.uint8))
    _check(lib.gs_layout_host(rp.ctypes.data, n, t.ctypes.data, w.ctypes.data, t.shape[0], vocab, prec,
                              ctypes.addressof(padded), out["term_off"].ctypes.data, out["term_len"].ctypes.data,
                              out["post_doc"].ctypes.data, out["post_w"].ctypes.data, out["blk_max"].ctypes.data,
                              out["blk_first_doc"].ctypes.data, out["term_dense"].ctypes.data,
                              out["post_b8"].ctypes.data), "gs_layout_host")
    return out


def query_plan_host(precision, q_weights, term_max, term_min):
    """Per-query fixed-point plan (gs_query_plan_host): (F, abs_err bound, wide-range limit)."""
    w, a, b = _np(q_weights, np.float32), _np(term_max, np.float32), _np(term_min, np.float32)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    F, e, lim = ctypes.c_int32(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(lib.gs_query_plan_host(prec, w.ctypes.data, a.ctypes.data, b.ctypes.data, w.shape[0], ctypes.byref(F),
                                  ctypes.byref(e), ctypes.byref(lim)), "gs_query_plan_host")
    return int(F.value), float(e.value), float(lim.value)


class Index:
    """GPU-resident inverted index built from a doc-major CSR (row_ptr, terms, weights)."""

    def __init__(self, row_ptr, terms, weights, vocab: int, precision="fp32", keep_forward: bool = False,
                 stream=None, keep_doc_ids: bool = False):
        rp, t, w = _np(row_ptr, np.int64), _np(terms, np.int32), _np(weights, np.float32)
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        flags = (GS_KEEP_FORWARD if keep_forward else 0) | (GS_KEEP_DOC_IDS if keep_doc_ids else 0)
        h = ctypes.c_void_p()
        _check(lib.gs_build_index(rp.ctypes.data, rp.shape[0] - 1, t.ctypes.data, w.ctypes.data, t.shape[0], vocab,
                                  self.precision, flags, _stream_ptr(stream), ctypes.byref(h)), "gs_build_index")
        self._h = h
        self.vocab = vocab
        self._tuned = {}  # autotuner choices: (index handle, batch capacity, k_max) -> (best, table)

    @classmethod
    def from_rows(cls, rows, precision="fp32", keep_forward=False, stream=None, keep_doc_ids=False):
        return cls(rows.row_ptr, rows.terms, rows.weights, rows.vocab, precision, keep_forward, stream,
                   keep_doc_ids)

    @property
    def handle(self):
        return self._h

    def info(self) -> IndexInfo:
        i = IndexInfo()
        _check(lib.gs_index_info(self._h, ctypes.byref(i)), "gs_index_info")
        return i

    def dense_terms(self) -> np.ndarray:
        """uint8 [vocab]: 1 where the term's doc ids have the byte form (every 64-block spans <= 256 docs)."""
        v = self.info().vocab_size
        out = np.zeros(v, dtype=np.uint8)
        _check(lib.gs_index_dense_terms(self._h, out.ctypes.data, v), "gs_index_dense_terms")
        return out

    @property
    def n_docs(self) -> int:
        return int(self.info().n_docs)

    def workspace_bytes(self, query_tile: int, opts: Optional[SearchOpts] = None) -> int:
        n = ctypes.c_size_t(0)
        _check(lib.gs_workspace_size(self._h, int(query_tile), ctypes.byref(opts) if opts else None,
                                     ctypes.byref(n)), "gs_workspace_size")
        return int(n.value)

    def search_workspace_bytes(self, n_queries: int, q_nnz: int, k_max: int, opts: Optional[SearchOpts] = None) -> int:
        n = ctypes.c_size_t(0)
        _check(lib.gs_search_workspace_size(self._h, int(n_queries), int(q_nnz), int(k_max),
                                            ctypes.byref(opts) if opts else None, ctypes.byref(n)),
               "gs_search_workspace_size")
        return int(n.value)

    def workspace(self, query_tile: int, opts: Optional[SearchOpts] = None, device="cuda") -> torch.Tensor:
        return torch.empty(self.workspace_bytes(query_tile, opts), dtype=torch.uint8, device=device)

    def batch(self, queries, k, k_max: Optional[int] = None, stream=None) -> "Batch":
        return Batch(self, queries.row_ptr, queries.terms, queries.weights, k, k_max, stream)

    def search(self, batch: "Batch", workspace: Optional[torch.Tensor] = None, opts: Optional[SearchOpts] = None,
               out=None, stream=None):
        """Exact top-k of a prepared batch. Returns (ids [n, k_max] int32, scores [n, k_max]) on the device."""
        own_ws = workspace is None
        if own_ws:
            workspace = self.workspace(max(1, min(batch.n_queries, 64)), opts)
        if out is None:
            ids = torch.empty((batch.n_queries, batch.k_max), dtype=torch.int32, device=workspace.device)
            scores = torch.empty((batch.n_queries, batch.k_max), dtype=SCORE_DTYPES[self.precision],
                                 device=workspace.device)
        else:
            ids, scores = out
        _check(lib.gs_search_batch(self._h, batch.handle, workspace.data_ptr(), workspace.numel(), ids.data_ptr(),
                                   scores.data_ptr(), ctypes.byref(opts) if opts else None, _stream_ptr(stream)),
               "gs_search_batch")
        if own_ws and stream is not None:
            # the implicit workspace is freed on return while the search may still run on `stream`
            workspace.record_stream(stream)
        return ids, scores

    def search_noalloc(self, batch: "Batch", out, opts: Optional[SearchOpts] = None, stream=None):
        """gs_search_batch_noalloc: the search with the library's fixed scratch array (no allocation)."""
        ids, scores = out
        _check(lib.gs_search_batch_noalloc(self._h, batch.handle, ids.data_ptr(), scores.data_ptr(),
                                           ctypes.byref(opts) if opts else None, _stream_ptr(stream)),
               "gs_search_batch_noalloc")
        return ids, scores

    def search_host(self, queries, k, k_max: Optional[int] = None, workspace: Optional[torch.Tensor] = None,
                    opts: Optional[SearchOpts] = None, stream=None):
        """gs_search: host CSR in, synchronous."""
        rp, t, w = _np(queries.row_ptr, np.int64), _np(queries.terms, np.int32), _np(queries.weights, np.float32)
        nq = rp.shape[0] - 1
        kk = np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)).copy()
        k_max = int(kk.max()) if k_max is None and nq else int(k_max or 0)
        if workspace is None:
            workspace = self.workspace(max(1, min(nq, 64)), opts)
        ids = torch.empty((nq, k_max), dtype=torch.int32, device=workspace.device)
        scores = torch.empty((nq, k_max), dtype=SCORE_DTYPES[self.precision], device=workspace.device)
        _check(lib.gs_search(self._h, rp.ctypes.data, nq, t.ctypes.data, w.ctypes.data, t.shape[0], kk.ctypes.data,
                             k_max, workspace.data_ptr(), workspace.numel(), ids.data_ptr(), scores.data_ptr(),
                             ctypes.byref(opts) if opts else None, _stream_ptr(stream)), "gs_search")
        return ids, scores

    def autotune(self, batch: "Batch", workspace: Optional[torch.Tensor] = None, reps: int = 2, stream=None,
                 cache: bool = True, return_outputs: bool = False):
        """Time every candidate option set on this batch; returns (best SearchOpts, [(opts dict, ms), ...]),
        plus (ids, scores) as numpy arrays (the best option set's result) with return_outputs.

        With cache, the choice is kept per (index, batch capacity, k_max) for the life of the index.
        """
        key = (self._h.value, batch.n_queries, batch.k_max)
        if cache and not return_outputs and key in self._tuned:
            return self._tuned[key]
        if workspace is None:
            workspace = self.workspace(batch.n_queries)
        ids = torch.empty((batch.n_queries, batch.k_max), dtype=torch.int32, device=workspace.device)
        sc = torch.empty((batch.n_queries, batch.k_max), dtype=SCORE_DTYPES[self.precision], device=workspace.device)
        best = SearchOpts()
        cands = (SearchOpts * 64)()
        times = (ctypes.c_float * 64)()
        n = ctypes.c_int32(0)
        _check(lib.gs_autotune(self._h, batch.handle, workspace.data_ptr(), workspace.numel(), ids.data_ptr(),
                               sc.data_ptr(), int(reps), _stream_ptr(stream), ctypes.byref(best), cands, times, 64,
                               ctypes.byref(n)), "gs_autotune")
        table = [({"kernel": cands[i].kernel, "tile_docs": cands[i].tile_docs, "chunk": cands[i].chunk},
                  float(times[i])) for i in range(min(n.value, 64))]
        if cache:
            self._tuned[key] = (best, table)
        if return_outputs:
            return best, table, (ids.cpu().numpy(), sc.cpu().numpy())
        return self._tuned[key] if cache else (best, table)

    def close(self):
        if getattr(self, "_h", None):
            lib.gs_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A validated query batch resident on the device (capacity = its query count unless reserved)."""

    def __init__(self, index: Index, row_ptr, terms, weights, k, k_max=None, stream=None):
        rp, t, w = _np(row_ptr, np.int64), _np(terms, np.int32), _np(weights, np.float32)
        nq = rp.shape[0] - 1
        kk = np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)).copy()
        self.k = kk
        self.k_max = int(kk.max()) if k_max is None and nq else int(k_max or 0)
        self.n_queries = nq
        h = ctypes.c_void_p()
        _check(lib.gs_batch_create(index.handle, rp.ctypes.data, nq, t.ctypes.data, w.ctypes.data, t.shape[0],
                                   kk.ctypes.data, self.k_max, _stream_ptr(stream), ctypes.byref(h)),
               "gs_batch_create")
        self._h = h
        self._index = index

    @classmethod
    def reserve(cls, index: Index, max_queries: int, max_nnz: int, k_max: int) -> "Batch":
        self = cls.__new__(cls)
        h = ctypes.c_void_p()
        _check(lib.gs_batch_reserve(index.handle, int(max_queries), int(max_nnz), int(k_max), ctypes.byref(h)),
               "gs_batch_reserve")
        self._h, self._index = h, index
        self.n_queries, self.k_max = int(max_queries), int(k_max)
        self.k = np.zeros(self.n_queries, np.int32)
        return self

    def update(self, queries, k, stream=None):
        """Refill in place (at most the reserved capacity); unused slots become empty queries with k = 0."""
        rp, t, w = _np(queries.row_ptr, np.int64), _np(queries.terms, np.int32), _np(queries.weights, np.float32)
        nq = rp.shape[0] - 1
        kk = np.broadcast_to(np.asarray(k, dtype=np.int32), (nq,)).copy()
        _check(lib.gs_batch_update(self._h, rp.ctypes.data, nq, t.ctypes.data, w.ctypes.data, t.shape[0],
                                   kk.ctypes.data, _stream_ptr(stream)), "gs_batch_update")
        self.k = np.zeros(self.n_queries, np.int32)
        self.k[:nq] = kk

    @property
    def handle(self):
        return self._h

    def diagnostics(self) -> np.ndarray:
        """[n_queries, 8]: candidates, refinement passes, bf16 band size, overflow flag, rows scored
        again (0 no, 1 fused-filtering fallback, 2 wide range: fp64 pass), fused filtering used,
        64-posting blocks skipped by pruning, 0."""
        out = np.zeros((self.n_queries, 8), dtype=np.int32)
        _check(lib.gs_batch_diagnostics(self._h, out.ctypes.data), "gs_batch_diagnostics")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib.gs_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured search (hipGraph) bound to an index, a batch, a workspace and output tensors."""

    def __init__(self, index: Index, batch: Batch, workspace: torch.Tensor, ids: torch.Tensor, scores: torch.Tensor,
                 opts: Optional[SearchOpts] = None, stream=None):
        h = ctypes.c_void_p()
        _check(lib.gs_graph_create(index.handle, batch.handle, workspace.data_ptr(), workspace.numel(),
                                   ids.data_ptr(), scores.data_ptr(), ctypes.byref(opts) if opts else None,
                                   _stream_ptr(stream), ctypes.byref(h)), "gs_graph_create")
        self._h = h
        self._keep = (index, batch, workspace, ids, scores)

    def launch(self, stream=None):
        _check(lib.gs_graph_launch(self._h, _stream_ptr(stream)), "gs_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            lib.gs_graph_free(self._h)
            self._h = None
        self._keep = None  # releases the buffers the graph was bound to

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (gs_server_*) over a resident index; admission by memory_budget."""

    def __init__(self, index: Index, max_batch: int = 32, n_slots: int = 4, k_max: int = 1000, memory_budget: int = 0,
                 opts: Optional[SearchOpts] = None):
        o = ServerOpts()
        o.max_batch, o.n_slots, o.k_max, o.memory_budget = int(max_batch), int(n_slots), int(k_max), int(memory_budget)
        if opts is not None:
            o.search = opts
        h = ctypes.c_void_p()
        _check(lib.gs_server_create(index.handle, ctypes.byref(o), ctypes.byref(h)), "gs_server_create")
        self._h, self._index = h, index
        self.k_max = int(k_max)
        self.score_dtype = {GS_FP32: np.float32, GS_BF16: np.float64, GS_U8: np.int32}[index.precision]

    def submit(self, terms, weights, k: int) -> int:
        t, w = _np(terms, np.int32), _np(weights, np.float32)
        r = lib.gs_server_submit(self._h, t.ctypes.data, w.ctypes.data, t.shape[0], int(k))
        if r < 0:
            raise GsError(int(r), "gs_server_submit", lib.gs_last_error().decode())
        return int(r)

    def wait(self, ticket: int, k: int, timeout_ms: int = -1):
        """(ids [k] int32, scores [k], latency ms) of a submitted query."""
        ids = np.empty(max(k, 1), np.int32)
        sc = np.empty(max(k, 1), self.score_dtype)
        lat = ctypes.c_double(0)
        _check(lib.gs_server_wait(self._h, int(ticket), int(timeout_ms), ids.ctypes.data, sc.ctypes.data,
                                  ctypes.byref(lat)), "gs_server_wait")
        return ids[:k], sc[:k], lat.value

    def poll(self, ticket: int, k: int):
        """(ids, scores, latency ms) if the query has finished, else None (gs_server_poll)."""
        ids = np.empty(max(k, 1), np.int32)
        sc = np.empty(max(k, 1), self.score_dtype)
        lat = ctypes.c_double(0)
        rc = lib.gs_server_poll(self._h, int(ticket), ids.ctypes.data, sc.ctypes.data, ctypes.byref(lat))
        if rc == GS_ETIMEOUT:
            return None
        _check(rc, "gs_server_poll")
        return ids[:k], sc[:k], lat.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib.gs_server_stats(self._h, ctypes.byref(s)), "gs_server_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib.gs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_fail_alloc(n: int):
    """Test hook: the library's allocation after n more succeeds fails once (n < 0 disarms)."""
    lib.gs_debug_fail_alloc(int(n))


def version() -> str:
    return lib.gs_version().decode()


def device_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """Plain 16-byte-vector copy (traffic-counter yardstick)."""
    n = min(dst.numel() * dst.element_size(), src.numel() * src.element_size())
    _check(lib.gs_device_copy(dst.data_ptr(), src.data_ptr(), n, _stream_ptr(stream)), "gs_device_copy")


LDS_ATOMIC_OPS = {"u32": 0, "u64": 1, "f32": 2, "f64": 3}


def lds_atomic_probe(op: str, pattern: int, workgroups: int, iters: int, sink: torch.Tensor, stream=None) -> int:
    """Launch the LDS atomic-add yardstick (asynchronous); returns the lane-ops it issues."""
    n = ctypes.c_int64(0)
    assert sink.numel() * sink.element_size() >= 8 * workgroups
    _check(lib.gs_lds_atomic_probe(LDS_ATOMIC_OPS[op], int(pattern), int(workgroups), int(iters), sink.data_ptr(),
                                   _stream_ptr(stream), ctypes.byref(n)), "gs_lds_atomic_probe")
    return int(n.value)


def timing_enable(on: bool = True):
    _check(lib.gs_timing_enable(1 if on else 0), "gs_timing_enable")


def timing_read():
    """{'score_ms', 'score_launches', 'select_ms', 'select_launches'} summed since the previous read."""
    a, c = ctypes.c_double(0), ctypes.c_double(0)
    b, d = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib.gs_timing_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)), "gs_timing_read")
    return {"score_ms": a.value, "score_launches": b.value, "select_ms": c.value, "select_launches": d.value}
