#!/usr/bin/env python3
"""Throughput of exact learned-sparse top-k retrieval on one MI355X.

Workload (default): 8.8M synthetic passages shaped like the paper's MS MARCO +
SPLADE collection (about 1.06 B postings), one batch of 500 queries, exact
top-1000 per query, fp32 posting weights. A step is one full search of the
batch (scoring + selection), with the index, the batch and the workspace
resident in HBM before the timed region starts.

Prints ONE JSON line (rank 0) with QPS, the roofline of the dominant kernel
(scoring; HIP events around its launches, algorithmic bytes = the postings of
every query term plus one write of each score array), the CPU oracle baseline
on a bounded sample of the same batch, and the other precision forms.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPS @8.8M docs top-1000 (fp32 vs uint8/bf16, batched); HBM GB/s %; p50/p99 ms"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
WEIGHT_BYTES = {"fp32": 4, "bf16": 2, "u8": 1}
DTYPE = {"fp32": "f32", "bf16": "bf16+f64", "u8": "u8/i32"}
T0 = time.time()


def log(msg):
    print("[bench %6.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="full-8.8m")
    ap.add_argument("--n-docs", type=int, default=0, help="override the collection size")
    ap.add_argument("--batch", type=int, default=0, help="override the number of queries")
    ap.add_argument("--k", type=int, default=1000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "u8"])
    ap.add_argument("--kernel", default="tiled", choices=["tiled", "atomic", "docpar", "shared", "group"])
    ap.add_argument("--tile-docs", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--forms", default="u8,bf16,fp32:shared,u8:shared,bf16:shared,u8:group",
                    help="other precision[:kernel[:chunk[:prune]]] forms to time (comma list, or 'none')")
    ap.add_argument("--cpu-sample", type=int, default=16, help="queries timed on the CPU oracle (0 = skip)")
    ap.add_argument("--profile", action="store_true", help="main form only, no CPU leg (for profiler runs)")
    ap.add_argument("--lds-probe", action="store_true", help="only the LDS atomic-add yardstick (for profiler runs)")
    ap.add_argument("--no-fused", action="store_true", help="main form: scan every score row (no fused candidate filtering)")
    ap.add_argument("--batched", default="u8,bf16",
                    help="precisions for the 4,096-query uneven batch (autotuned, graph vs plain), or 'none'")
    ap.add_argument("--batched-queries", type=int, default=4096)
    ap.add_argument("--top10", type=int, default=1, help="also time every form at top-10 (1) or not (0)")
    ap.add_argument("--serving", default="200,800,2000,16000,20000", help="Poisson arrival rates (QPS) for the serving loop, or 'none'")
    ap.add_argument("--serving-seconds", type=float, default=30.0, help="duration of each rate up to 2000 QPS")
    ap.add_argument("--serving-seconds-high", type=float, default=10.0, help="duration of each rate above 2000 QPS")
    ap.add_argument("--serving-budget-gib", type=float, default=8.0,
                    help="device memory for the in-flight queries' score buffers (admission by memory)")
    ap.add_argument("--serving-precision", default="u8")
    ap.add_argument("--serving-batch", type=int, default=64, help="most queries per device step of the server")
    ap.add_argument("--serving-slots", type=int, default=4, help="device slots (concurrent steps) of the server")
    ap.add_argument("--serving-kernel", default="shared", choices=["tiled", "shared"], help="scoring kernel of the server")
    return ap.parse_args()


def algorithmic_bytes(df, queries, n_docs, wbytes, idbytes, written_docs=None):
    """Per-query postings of the query's terms (doc id + weight) and one score-array write / read.

    idbytes: bytes per posting for the doc id, a number or one per term. The doc-tiled
    kernels read a 16-bit doc offset (2), or with fp32/bf16 weights in the per-query
    kernel, for terms in byte form, 1 byte plus a 4-byte base per 64 postings; the
    global-atomic kernel reads the 32-bit doc id (4). With fused candidate filtering
    (fp32, uint8) only the seed tiles' scores are written (written_docs per query).
    """
    p_q = np.array([int(df[queries.row(i)[0]].sum()) for i in range(queries.n_rows)], dtype=np.int64)
    per_term = df * (np.broadcast_to(np.asarray(idbytes, dtype=np.float64), df.shape) + wbytes)
    post_bytes = sum(float(per_term[queries.row(i)[0]].sum()) for i in range(queries.n_rows))
    wd = n_docs if written_docs is None else written_docs
    score_kernel = int(round(post_bytes)) + queries.n_rows * wd * 4
    step = score_kernel + queries.n_rows * wd * 4  # the filter reads what was written
    return p_q, score_kernel, step


_C_TOKEN = re.compile(r'//[^\n]*|/\*.*?\*/|"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'', re.S)


def survey_model_bytes(p_q, n_docs, wbytes):
    """The per-query byte model of the scope table: P_q * (4 + s_w) + 8 N (postings with a 4-byte doc id and
    an s_w-byte weight, one write and one read of the 4-byte score array), summed over the queries."""
    return int(np.sum(p_q.astype(np.float64) * (4 + wbytes)) + p_q.shape[0] * 8 * n_docs)


def code_digest(files):
    """sha256 of C/HIP sources with comments removed and whitespace collapsed.

    A comment edit leaves it unchanged; any change to the code itself changes it.
    """
    import hashlib
    h = hashlib.sha256()
    for f in files:
        src = open(os.path.join(ROOT, f)).read()
        src = _C_TOKEN.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def profiled_traffic(kernel, precision, workload_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if the kernel code is unchanged."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        meta = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if (meta.get("kernel"), meta.get("precision"), meta.get("workload")) != (kernel, precision, workload_name):
            continue
        if code_digest(meta["source_files"]) == meta["code_sha256"]:
            return int(meta["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def score_error(oracle, docs, queries, s, k, rid, results):
    """Error of each precision against the exact fp64 scores, on the first s queries.

    fp32: relative error of the returned scores. u8: recall of the fp64 top-k and the
    relative error of the dequantised impact score S8/85^2. bf16: the returned scores are
    fp64-rescored (exact); the error before rescoring is that of bf16-rounded posting
    weights, evaluated exactly on the returned docs.
    """
    import workload

    out = {}
    for prec, res in results:
        if prec in out:
            continue
        rel, recall = [], []
        if prec == "bf16":
            u = docs.weights.view(np.uint32).astype(np.uint64)
            u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
            rounded = workload.SparseRows(docs.row_ptr, docs.terms, u.view(np.float32), docs.vocab)
        for q in range(s):
            t_, w_ = queries.row(q)
            kq = min(int(k), docs.n_rows)
            ids = np.asarray(res["ids"][q][:kq])
            exact, _ = oracle.pair_scores(docs, t_, w_, ids)
            nz = exact > 0
            if prec == "fp32":
                got = np.asarray(res["scores"][q][:kq], dtype=np.float64)
            elif prec == "u8":
                got = np.asarray(res["scores"][q][:kq], dtype=np.float64) / 7225.0
                recall.append(len(set(ids.tolist()) & set(np.asarray(rid[q][:kq]).tolist())) / kq)
            else:
                got, _ = oracle.pair_scores(rounded, t_, w_, ids)
            rel.append(np.abs(got[nz] - exact[nz]) / exact[nz])
        rel = np.concatenate(rel) if rel else np.zeros(0)
        e = {"queries": s, "results": int(rel.size),
             "rel_err_max": float("%.3g" % rel.max()) if rel.size else 0.0,
             "rel_err_mean": float("%.3g" % rel.mean()) if rel.size else 0.0}
        if prec == "u8":
            e["what"] = "dequantised int32 score S8/85^2 vs exact fp64 score"
            e["recall_at_k_mean"] = round(float(np.mean(recall)), 4)
            e["recall_at_k_min"] = round(float(np.min(recall)), 4)
        elif prec == "bf16":
            e["what"] = "before fp64 rescoring (bf16-rounded posting weights); returned scores are exact"
        else:
            e["what"] = "returned fp32 score vs exact fp64 score"
        out[prec] = e
    return out


CU_COUNT, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock


def lds_atomic_rates(gs, torch, workgroups=2048, iters=1024, reps=5):
    """LDS atomic-add throughput per accumulator type (lane-ops per clock per CU at 2.4 GHz)."""
    sink = torch.empty(workgroups * 8, dtype=torch.uint8, device="cuda")
    out = {}
    for op in ("u32", "u64", "f32", "f64"):
        for pattern, pname in ((0, "scattered"), (1, "consecutive")):
            gs.lds_atomic_probe(op, pattern, workgroups, iters, sink)  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            n = 0
            for _ in range(reps):
                n += gs.lds_atomic_probe(op, pattern, workgroups, iters, sink)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            out["%s_%s" % (op, pname)] = round(n / (ms / 1e3) / CU_COUNT / CLOCK_HZ, 3)
    out["unit"] = "lane-ops per clock per CU (%d CUs at %.1f GHz), %d x 512 lanes x %d adds into 64 KiB of LDS" % (
        CU_COUNT, CLOCK_HZ / 1e9, workgroups, iters)
    return out


class IndexCache:
    """One resident index per (precision, forward rows kept, 32-bit doc ids kept), built on first use:
    the document-parallel kernel needs the forward rows, the global-atomic kernel the doc ids."""

    def __init__(self, gs, docs):
        self.gs, self.docs, self.idx = gs, docs, {}

    def get(self, precision, kernel="tiled"):
        key = (precision, kernel == "docpar" or precision == "bf16", kernel == "atomic")
        if key not in self.idx:
            log("index %s%s%s ..." % (precision, " + forward rows" if key[1] else "", " + doc ids" if key[2] else ""))
            self.idx[key] = self.gs.Index.from_rows(self.docs, precision, keep_forward=key[1], keep_doc_ids=key[2])
        return self.idx[key]

    def drop(self, precision):
        for key in [k for k in self.idx if k[0] == precision]:
            self.idx.pop(key).close()


def time_form(gs, torch, idx, queries, k, opts, steps, warmup, host_steps=0):
    batch = idx.batch(queries, k)
    nq = queries.n_rows
    ws = idx.workspace(nq, opts)
    ids = torch.empty((nq, batch.k_max), dtype=torch.int32, device="cuda")
    sc = torch.empty((nq, batch.k_max), dtype=gs.SCORE_DTYPES[idx.precision], device="cuda")
    for _ in range(warmup):
        idx.search(batch, ws, opts, out=(ids, sc))
    torch.cuda.synchronize()
    gs.timing_read()
    gs.timing_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        idx.search(batch, ws, opts, out=(ids, sc))
        ev[i + 1].record()
    torch.cuda.synchronize()
    gs.timing_enable(False)
    t = gs.timing_read()
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    total_ms = ev[0].elapsed_time(ev[steps])
    diag = batch.diagnostics()
    res = {"ids": ids.cpu().numpy(), "scores": sc.cpu().numpy(), "total_ms": total_ms, "step_ms": step_ms,
           "timing": t, "diag": diag, "device_bytes": int(idx.info().device_bytes), "ws_bytes": ws.numel(),
           "dense_terms": idx.dense_terms()}
    if host_steps:
        # host CSR in (validation, per-query scales, upload), results copied back to host memory
        host_ms = []
        for _ in range(host_steps):
            t0 = time.perf_counter()
            hi, hs = idx.search_host(queries, k, workspace=ws, opts=opts)
            hi, hs = hi.cpu().numpy(), hs.cpu().numpy()
            host_ms.append((time.perf_counter() - t0) * 1e3)
            assert np.array_equal(hi, res["ids"]) and np.array_equal(hs, res["scores"]), "host-CSR search differs"
        res["host_ms"] = np.array(host_ms)
    del ws, ids, sc
    batch.close()
    torch.cuda.empty_cache()
    return res


def run_batched(gs, torch, docs, args, indexes):
    """Uneven batch: lognormal query lengths (median 25, 5..250), k mixed over {10, 100, 1000}; autotuned
    options; one persistent-or-grid launch per step; hipGraph replay vs plain launches; oracle-checked sample."""
    import workload
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_rules import check_exact_f64, check_exact_int

    w = workload.WORKLOADS["uneven-8.8m"]
    nq = args.batched_queries
    queries = workload.make_queries(w, n=nq)
    k = workload.k_mix(nq, seed=4)
    res = {"workload": w.name, "queries": nq, "query_nnz_mean": round(queries.nnz / nq, 2),
           "query_nnz_max": int(np.diff(queries.row_ptr).max()), "k_mix": [10, 100, 1000]}
    threads = host_threads()["threads"]
    for prec in [p for p in args.batched.split(",") if p]:
        idx = indexes.get(prec)
        log("batched %s: autotune ..." % prec)
        tune_q = queries.subset(np.arange(min(512, nq)))
        tb = idx.batch(tune_q, k[: tune_q.n_rows], k_max=1000)
        best, table = idx.autotune(tb, reps=1)
        tb.close()
        opts = gs.make_opts(best.kernel, tile_docs=best.tile_docs, chunk=best.chunk)
        batch = idx.batch(queries, k, k_max=1000)
        ws = idx.workspace(nq, opts)
        ids = torch.empty((nq, 1000), dtype=torch.int32, device="cuda")
        sc = torch.empty((nq, 1000), dtype=gs.SCORE_DTYPES[idx.precision], device="cuda")
        idx.search(batch, ws, opts, out=(ids, sc))
        torch.cuda.synchronize()
        steps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            idx.search(batch, ws, opts, out=(ids, sc))
        e1.record()
        torch.cuda.synchronize()
        plain_ms = e0.elapsed_time(e1) / steps
        graph = gs.Graph(idx, batch, ws, ids, sc, opts)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            graph.launch()
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / steps
        diag = batch.diagnostics()
        got_ids, got_sc = ids.cpu().numpy(), sc.cpu().numpy()
        graph.close()
        del graph, ws, ids, sc
        torch.cuda.empty_cache()
        # small batch (16 queries): where launch overhead matters
        small = queries.subset(np.arange(16))
        sb = idx.batch(small, k[:16], k_max=1000)
        sws = idx.workspace(16, opts)
        sids = torch.empty((16, 1000), dtype=torch.int32, device="cuda")
        ssc = torch.empty((16, 1000), dtype=gs.SCORE_DTYPES[idx.precision], device="cuda")
        idx.search(sb, sws, opts, out=(sids, ssc))
        g16 = gs.Graph(idx, sb, sws, sids, ssc, opts)
        torch.cuda.synchronize()
        reps = 20
        e0.record()
        for _ in range(reps):
            idx.search(sb, sws, opts, out=(sids, ssc))
        e1.record()
        torch.cuda.synchronize()
        small_plain = e0.elapsed_time(e1) / reps
        e0.record()
        for _ in range(reps):
            g16.launch()
        e1.record()
        torch.cuda.synchronize()
        small_graph = e0.elapsed_time(e1) / reps
        g16.close()
        # oracle-checked sample of the large batch
        s = 4
        sample = queries.subset(np.arange(s))
        status = "ok"
        try:
            if prec == "u8":
                rid, rsc = oracle.topk_i64(docs, sample, k[:s], k_max=1000, n_threads=threads)
                for q in range(s):
                    check_exact_int(got_ids[q], got_sc[q], rid[q], rsc[q], what="batched u8")
            else:
                rid, rsc = oracle.topk_f64(docs, sample, k[:s], k_max=1000, n_threads=threads)
                for q in range(s):
                    check_exact_f64(got_ids[q], got_sc[q], rid[q], rsc[q], what="batched bf16")
            status = "exact on %d sampled queries" % s
        except AssertionError as e:
            status = "MISMATCH: " + str(e)[:160]
        names = {v: k for k, v in gs.KERNELS.items()}
        res[prec] = {"qps_plain": round(nq / (plain_ms / 1e3), 1), "qps_graph": round(nq / (graph_ms / 1e3), 1),
                     "ms_plain": round(plain_ms, 3), "ms_graph": round(graph_ms, 3),
                     "small_batch_16": {"ms_plain": round(small_plain, 3), "ms_graph": round(small_graph, 3)},
                     "tuned": {"kernel": names.get(best.kernel, best.kernel), "tile_docs": best.tile_docs,
                               "chunk": best.chunk},
                     "tuning_table_ms": [[names.get(c["kernel"], c["kernel"]), c["tile_docs"], c["chunk"],
                                          round(t, 2)] for c, t in table],
                     "overflow": int(diag[:, 3].max()), "parity": status}
        log("batched %s: plain %.1f QPS, graph %.1f QPS, tuned %s; %s" % (prec, res[prec]["qps_plain"],
                                                                         res[prec]["qps_graph"], res[prec]["tuned"],
                                                                         status))
        sb.close()
        batch.close()
        del g16, sws, sids, ssc
        torch.cuda.empty_cache()
    return res


def run_serving(gs, torch, docs, args, indexes):
    """Poisson arrivals into the continuous-batching loop; latency = submission to results on the host.

    Admission is by memory: the server's workspace arena holds as many query rows (score array plus
    selection scratch) as the budget allows. The first requests of the first rate are checked
    against the oracle."""
    import threading
    import oracle
    import workload
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity_rules import check_exact_f64, check_exact_int

    prec = args.serving_precision
    idx = indexes.get(prec)
    pool = workload.queries_lognormal(8192, seed=91)
    ks = workload.k_mix(8192, seed=92)
    max_batch, n_slots = args.serving_batch, args.serving_slots
    budget = int(args.serving_budget_gib * (1 << 30))
    srv = gs.Server(idx, max_batch=max_batch, n_slots=n_slots, k_max=1000, memory_budget=budget,
                    opts=gs.make_opts(args.serving_kernel))
    st = srv.stats()
    res = {"precision": prec, "kernel": args.serving_kernel, "max_batch": max_batch, "n_slots": n_slots,
           "memory_budget": budget, "arena_rows": st["arena_rows"], "row_bytes": st["row_bytes"],
           "query_law": "lognormal median 25, sigma 0.8, [5, 250]; k over {10, 100, 1000}"}
    for q in range(64):  # warm-up
        t, w = pool.row(q)
        srv.wait(srv.submit(t, w, int(ks[q])), int(ks[q]))
    sample = {}
    for ri, rate in enumerate([float(r) for r in args.serving.split(",") if r]):
        secs = args.serving_seconds if rate <= 2000 else args.serving_seconds_high
        arrivals = workload.poisson_arrivals(rate, secs, seed=int(rate))
        n = arrivals.shape[0]
        tickets = [None] * n
        lat = np.zeros(n)
        done_at = np.zeros(n)
        keep = 8 if ri == 0 else 0

        def collector():
            for i in range(n):
                while tickets[i] is None:
                    time.sleep(1e-5)
                kq = int(ks[i % 8192])
                ids_i, sc_i, lat[i] = srv.wait(tickets[i], kq)
                done_at[i] = time.perf_counter()
                if i < keep:
                    sample[i] = (ids_i.copy(), sc_i.copy())

        before = srv.stats()
        th = threading.Thread(target=collector)
        th.start()
        t0 = time.perf_counter()
        for i in range(n):
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            t, w = pool.row(i % 8192)
            tickets[i] = srv.submit(t, w, int(ks[i % 8192]))
        th.join()
        span = max(done_at.max() - t0, secs)
        after = srv.stats()
        steps = after["device_steps"] - before["device_steps"]
        res["rate_%d" % int(rate)] = {
            "offered_qps": rate, "seconds": secs, "requests": n, "sustained_qps": round(n / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_batch": round((after["completed"] - before["completed"]) / max(steps, 1), 2),
            "max_in_flight": after["max_in_flight"], "failed": after["failed"] - before["failed"]}
        log("serving %s @%d QPS for %.0f s: sustained %.1f, p50 %.2f ms, p99 %.2f ms, mean batch %.1f"
            % (prec, rate, secs, n / span, np.percentile(lat, 50), np.percentile(lat, 99),
               res["rate_%d" % int(rate)]["mean_batch"]))
    srv.close()
    # oracle check of the first served requests (same queries, same k)
    if sample:
        s = len(sample)
        sub = pool.subset(np.arange(s))
        kk = ks[:s]
        threads = host_threads()["threads"]
        try:
            if prec == "u8":
                rid, rsc = oracle.topk_i64(docs, sub, kk, k_max=1000, n_threads=threads)
                for i in range(s):
                    check_exact_int(sample[i][0], sample[i][1], rid[i][:kk[i]], rsc[i][:kk[i]], what="served")
                res["parity"] = "bit-exact on the first %d served requests" % s
            elif prec == "bf16":
                rid, rsc = oracle.topk_f64(docs, sub, kk, k_max=1000, n_threads=threads)
                for i in range(s):
                    check_exact_f64(sample[i][0], sample[i][1], rid[i][:kk[i]], rsc[i][:kk[i]], what="served")
                res["parity"] = "ids and fp64 scores identical on the first %d served requests" % s
        except AssertionError as e:
            res["parity"] = "MISMATCH: " + str(e)[:160]
        log("serving parity: %s" % res.get("parity"))
    torch.cuda.empty_cache()
    return res


def host_threads():
    """Host CPUs for the oracle: the process's affinity set, capped by OMP_NUM_THREADS when it is set
    (a shared GPU machine gives each GPU a CPU share and sets it)."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"threads": min(aff, omp) if omp > 0 else aff, "affinity_cpus": aff, "nproc": os.cpu_count(),
            "omp_num_threads": omp or None, "cpu_model": model}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    import workload
    import paper_2606_26441_amd as gs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.lds_probe:
        print(json.dumps({"lds_atomic": lds_atomic_rates(gs, torch)}), flush=True)
        return
    w = workload.WORKLOADS[args.workload]
    n_docs = args.n_docs or w.n_docs
    nq = args.batch or w.n_queries
    log("synthesising %d docs (%s) ..." % (n_docs, w.name))
    docs = workload.make_collection(w, n_docs=n_docs)
    queries = workload.make_queries(w, n=nq)
    log("collection: %d postings; queries: %d (mean nnz %.1f)" % (docs.nnz, nq, queries.nnz / max(nq, 1)))
    df = np.bincount(docs.terms, minlength=docs.vocab)
    opts = gs.make_opts(args.kernel, tile_docs=args.tile_docs, chunk=args.chunk, fused_filter=not args.no_fused)
    indexes = IndexCache(gs, docs)

    # yardstick: a plain 2 GiB device copy (reads and writes exactly its size once)
    src = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    gs.device_copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        gs.device_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log("device copy yardstick: %.0f GB/s (read + write)" % copy_gbs)
    lds_rates = None if args.profile else lds_atomic_rates(gs, torch)
    if lds_rates:
        log("LDS atomic yardstick: %s" % lds_rates)

    log("main form: %s / %s, %d warmup + %d timed steps" % (args.precision, args.kernel, args.warmup, args.steps))
    main_idx = indexes.get(args.precision, args.kernel)
    main_res = time_form(gs, torch, main_idx, queries, args.k, opts, args.steps, args.warmup,
                         host_steps=0 if args.profile else 3)
    written = None
    tile_docs = args.tile_docs or (8192 if args.precision == "fp32" else 16384)
    n_tiles = (n_docs + tile_docs - 1) // tile_docs
    if (not args.no_fused and args.kernel in ("tiled", "shared", "group") and nq >= 32
            and args.k <= 1024 and n_tiles >= 16):
        # fused candidate filtering: score rows of the seed tiles (every 8th) only
        written = sum(min(tile_docs, n_docs - t * tile_docs) for t in range(0, n_tiles, 8))
    if args.kernel == "tiled" and args.precision != "u8":
        idbytes = np.where(main_res["dense_terms"] != 0, 1.0 + 4.0 / 64.0, 2.0)
    else:
        idbytes = 2 if args.kernel in ("tiled", "shared", "group") else 4
    p_q, layout_bytes, step_bytes = algorithmic_bytes(df, queries, n_docs, WEIGHT_BYTES[args.precision], idbytes,
                                                      written)
    survey_bytes = survey_model_bytes(p_q, n_docs, WEIGHT_BYTES[args.precision])
    if args.kernel == "docpar":
        # document-parallel: every forward row (term id + fp32 weight) per query, plus one score write
        layout_bytes = nq * (docs.nnz * 8 + n_docs * 4)
        survey_bytes = nq * (docs.nnz * 8 + n_docs * 4)
        step_bytes = layout_bytes + nq * n_docs * 4
    ms_per_step = main_res["total_ms"] / args.steps
    qps = nq * args.steps / (main_res["total_ms"] / 1e3)
    t = main_res["timing"]
    score_ms = t["score_ms"] / max(t["score_launches"], 1)
    select_ms = t["select_ms"] / max(t["select_launches"], 1)
    achieved = survey_bytes / (score_ms / 1e3) / 1e9
    layout_gbs = layout_bytes / (score_ms / 1e3) / 1e9
    log("QPS %.1f  ms/step %.2f  score %.2f ms  select %.2f ms  scoring: %.0f GB/s effective (model bytes), "
        "%.0f GB/s on its layout bytes" % (qps, ms_per_step, score_ms, select_ms, achieved, layout_gbs))

    kernel_name = {"tiled": "k_score_tiled", "shared": "k_score_persistent", "atomic": "k_score_atomic",
                   "docpar": "k_score_docpar", "group": "k_score_group"}[args.kernel]
    traffic, traffic_src = (None, None)
    if args.n_docs in (0, w.n_docs) and nq == w.n_queries and args.k == 1000 and not args.no_fused \
            and not args.tile_docs and not args.chunk:
        traffic, traffic_src = profiled_traffic(kernel_name, args.precision, w.name)
    out = {
        "metric": METRIC,
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded Zipf(1.1)/Poisson/lognormal stand-in for MS MARCO + SPLADE)",
        "config": {"workload": w.name, "n_docs": n_docs, "postings": docs.nnz, "batch": nq, "k": args.k,
                   "precision": args.precision, "kernel": args.kernel, "tile_docs": tile_docs,
                   "chunk": args.chunk or 1024, "query_nnz_mean": round(queries.nnz / max(nq, 1), 2),
                   "postings_per_query_mean": int(p_q.mean())},
        "roofline": {
            "bound": "hbm", "kernel": kernel_name,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "frac_kind": "effective: the per-query model bytes P_q*(4+s_w) + 8N (postings with 4 B doc ids, one "
                         "score write and read) over the scoring launches' time; above 1 when the kernel moves "
                         "fewer bytes than the model (2- or 1-byte doc ids, score rows of seed tiles only)",
            "algorithmic_bytes_per_launch": survey_bytes,
            "layout_bytes_per_launch": layout_bytes,
            "layout_frac": round(layout_gbs / HBM_PEAK_GBS, 4),
            "hbm_frac_counters": None if traffic is None else round(traffic / (score_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                                                    4),
            "traffic_source": traffic_src,
            "launch_ms": round(score_ms, 4), "queries_per_launch": nq},
        "step": {"p50_ms": round(float(np.percentile(main_res["step_ms"], 50)), 3),
                 "p99_ms": round(float(np.percentile(main_res["step_ms"], 99)), 3),
                 "score_ms": round(score_ms, 3), "select_ms": round(select_ms, 3),
                 "hbm_frac_whole_step_layout": round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "memory": {"index_bytes": main_res["device_bytes"], "workspace_bytes": main_res["ws_bytes"]},
        "hbm_copy_GBs": round(copy_gbs, 1),
        "lds_atomic": lds_rates,
        "host_io": None if "host_ms" not in main_res else {
            "qps": round(nq / (float(np.median(main_res["host_ms"])) / 1e3), 2),
            "ms_per_batch": round(float(np.median(main_res["host_ms"])), 3),
            "what": "gs_search from a host CSR (validation + upload), results copied to host; median of %d"
                    % len(main_res["host_ms"])},
        "selection": {"candidates_mean": float(main_res["diag"][:, 0].mean()),
                      "refine_passes_max": int(main_res["diag"][:, 1].max()),
                      "overflow": int(main_res["diag"][:, 3].max()),
                      "wide_range_queries": int((main_res["diag"][:, 4] == 2).sum())},
    }

    main_name = args.precision if args.kernel == "tiled" else args.precision + ":" + args.kernel
    specs = []
    if not args.profile and args.forms != "none":
        for spec in [f for f in args.forms.split(",") if f]:
            parts = spec.split(":")
            prec, kern = parts[0], (parts[1] if len(parts) > 1 and parts[1] else "tiled")
            chunk = int(parts[2]) if len(parts) > 2 and parts[2] else 0
            prune = len(parts) > 3 and parts[3] == "prune"
            if (prec, kern, chunk, prune) != (args.precision, args.kernel, args.chunk, False):
                specs.append((prec, kern, chunk, prune))
    forms = {}
    for prec, kern, chunk, prune in specs:
        name = prec if kern == "tiled" else prec + ":" + kern
        name += (":%d" % chunk) if chunk else ""
        name += ":prune" if prune else ""
        log("form %s ..." % name)
        fsteps = max(3, args.steps // 2)
        r = time_form(gs, torch, indexes.get(prec, kern), queries, args.k,
                      gs.make_opts(kern, chunk=chunk, prune=prune), fsteps, 1)
        ms = r["total_ms"] / fsteps
        t = r["timing"]
        forms[name] = {"qps": round(nq / (ms / 1e3), 2), "ms_per_step": round(ms, 3),
                       "score_ms": round(t["score_ms"] / max(t["score_launches"], 1), 3),
                       "select_ms": round(t["select_ms"] / max(t["select_launches"], 1), 3),
                       "index_bytes": r["device_bytes"],
                       "overflow": int(r["diag"][:, 3].max())}
        if prune:
            forms[name]["pruned_blocks_per_query"] = round(float(r["diag"][:, 6].mean()), 1)
        forms[name]["_res"] = r
        log("form %s: QPS %.1f" % (name, forms[name]["qps"]))

    # top-10 of the same batch for every form (the paper's Fig. 1 cut-off), oracle-checked below
    top10 = {}
    if not args.profile and args.top10 and args.k != 10:
        for prec, kern, chunk, prune in [(args.precision, args.kernel, args.chunk, False)] + specs:
            name = prec if kern == "tiled" else prec + ":" + kern
            name += (":%d" % chunk) if chunk else ""
            name += ":prune" if prune else ""
            r = time_form(gs, torch, indexes.get(prec, kern), queries, 10,
                          gs.make_opts(kern, chunk=chunk, prune=prune), 3, 1)
            ms = r["total_ms"] / 3
            top10[name] = {"qps": round(nq / (ms / 1e3), 2), "ms_per_step": round(ms, 3), "_res": r}
            log("top-10 %s: QPS %.1f" % (name, top10[name]["qps"]))

    if not args.profile and args.cpu_sample > 0:
        import oracle
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity_rules import check_exact_f64, check_exact_int, check_fp32

        s = min(args.cpu_sample, nq)
        sample = queries.subset(np.arange(s))
        ht = host_threads()
        threads = ht["threads"]
        log("CPU oracle on %d queries with %d threads (%s) ..." % (s, threads, ht["cpu_model"]))
        t0 = time.time()
        rid, rsc = oracle.topk_f64(docs, sample, args.k, n_threads=threads)
        cpu_s = time.time() - t0
        out["cpu_baseline"] = {"value": round(s / cpu_s, 4), "unit": "queries/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "first %d of the %d queries, full %d-doc collection, exact fp64 top-%d "
                                         "with full sort; %.1f s wall" % (s, nq, n_docs, args.k, cpu_s),
                               "nproc": ht["nproc"], "affinity_cpus": ht["affinity_cpus"],
                               "omp_num_threads": ht["omp_num_threads"], "cpu_model": ht["cpu_model"]}
        t0 = time.time()
        oracle.topk_f64(docs, queries.subset(np.arange(1)), args.k, n_threads=1)
        out["cpu_single_thread"] = {"ms_per_query": round((time.time() - t0) * 1e3, 1),
                                    "sample": "the oracle on the first query, one thread"}
        log("CPU oracle, one thread: %.0f ms per query" % out["cpu_single_thread"]["ms_per_query"])

        def check(results, k, s_f, rid_f, rsc_f, s8, cache8):
            checked = {}
            try:
                for name, res in results:
                    prec = name.split(":")[0]
                    if prec == "fp32":
                        for q in range(s_f):
                            t_, w_ = queries.row(q)
                            check_fp32(docs, t_, w_, res["ids"][q], res["scores"][q], rid_f[q], rsc_f[q], k,
                                       what=name)
                        checked[name] = "within 1e-5, ids equal up to tolerance swaps (%d queries)" % s_f
                    elif prec == "bf16":
                        for q in range(s_f):
                            check_exact_f64(res["ids"][q], res["scores"][q], rid_f[q], rsc_f[q], what=name)
                        checked[name] = "ids and fp64 scores identical (%d queries)" % s_f
                    else:
                        if not cache8:
                            cache8.extend(oracle.topk_i64(docs, queries.subset(np.arange(s8)), k, n_threads=threads))
                        for q in range(s8):
                            check_exact_int(res["ids"][q], res["scores"][q], cache8[0][q], cache8[1][q], what=name)
                        checked[name] = "bit-exact (%d queries)" % s8
            except AssertionError as e:
                checked["error"] = str(e)[:200]
            return checked

        # full-size parity of the timed launch configurations on the same sample
        out["parity_sample"] = check([(main_name, main_res)] + [(n, f["_res"]) for n, f in forms.items()], args.k,
                                     s, rid, rsc, min(4, s), [])
        log("parity: %s" % out["parity_sample"])
        if top10:
            s10 = min(4, s)
            rid10, rsc10 = oracle.topk_f64(docs, queries.subset(np.arange(s10)), 10, n_threads=threads)
            chk10 = check([(n, f["_res"]) for n, f in top10.items()], 10, s10, rid10, rsc10, s10, [])
            for n in top10:
                top10[n]["parity"] = chk10.get(n, chk10.get("error"))
            log("top-10 parity: %s" % chk10)
        out["score_error"] = score_error(oracle, docs, queries, s, args.k, rid,
                                         [(args.precision, main_res)] + [(n.split(":")[0], f["_res"])
                                                                         for n, f in forms.items()])
        log("score error: %s" % out["score_error"])
    for f in list(forms.values()) + list(top10.values()):
        f.pop("_res", None)
    if forms:
        out["forms"] = forms
    if top10:
        out["top10"] = top10
    if not args.profile:
        indexes.drop("fp32")  # the batched and serving legs use the bf16 and uint8 indexes
        torch.cuda.empty_cache()
    if not args.profile and args.batched != "none":
        out["batched"] = run_batched(gs, torch, docs, args, indexes)
    if not args.profile and args.serving != "none":
        out["serving"] = run_serving(gs, torch, docs, args, indexes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
