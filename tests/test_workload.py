"""The seeded sampler: determinism, thread-count independence and the shape of its laws (CPU only)."""
import json
import os
import subprocess
import sys

import numpy as np

import oracle
import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_tiny_workload_digest_is_stable():
    g = json.load(open(os.path.join(GOLDEN, "workload_digests.json")))
    w = workload.WORKLOADS["tiny-10k"]
    assert workload.make_collection(w).digest() == g["docs"]
    assert workload.make_queries(w).digest() == g["queries"]


def test_thread_count_does_not_change_output():
    code = ("import workload; print(workload.collection(3000, seed=5).digest())")
    env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=os.path.dirname(GOLDEN) + "/..")
    one = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    assert one.stdout.strip() == workload.collection(3000, seed=5).digest()


def test_row_laws():
    docs = workload.collection(20000, seed=7)
    lens = np.diff(docs.row_ptr)
    assert lens.min() >= 8 and lens.max() <= 400
    assert abs(lens.mean() - 120) < 1.0
    for i in range(0, docs.n_rows, 997):
        t, w = docs.row(i)
        assert np.all(np.diff(t) > 0)  # distinct, ascending
    assert docs.weights.min() > 0 and docs.weights.max() <= 3.0
    df = np.bincount(docs.terms, minlength=workload.VOCAB)
    assert df.max() > 0.99 * docs.n_rows  # Zipf head terms occur in nearly every doc
    q = workload.queries_lognormal(4000, seed=9)
    ql = np.diff(q.row_ptr)
    assert ql.min() >= 5 and ql.max() <= 250 and 22 <= np.median(ql) <= 28


def test_stored_oracle_answers_for_tiny_workload():
    g = json.load(open(os.path.join(GOLDEN, "tiny10k_oracle.json")))
    w = workload.WORKLOADS["tiny-10k"]
    docs, qs = workload.make_collection(w), workload.make_queries(w)
    ids, sc = oracle.topk_f64(docs, qs, g["k"])
    assert ids.tolist() == g["f64_ids"]
    assert [[float(x).hex() for x in r] for r in sc] == g["f64_scores_hex"]
    ids8, sc8 = oracle.topk_i64(docs, qs, g["k"])
    assert ids8.tolist() == g["i64_ids"] and sc8.tolist() == g["i64_scores"]
