"""Writes the stored expected values under tests/golden/ (calls only workload/ and oracle/).

    python tests/golden/make_golden.py

* workload_digests.json - SHA-256 of the tiny 10K-doc workload arrays (a
  regression pin of the seeded sampler);
* tiny10k_oracle.json - the oracle's exact top-100 (fp64 and uint8-impact
  forms) for the 8 tiny-workload queries.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workload  # noqa: E402


def main():
    w = workload.WORKLOADS["tiny-10k"]
    docs = workload.make_collection(w)
    qs = workload.make_queries(w)
    json.dump({"workload": w.name, "docs": docs.digest(), "queries": qs.digest(),
               "docs_nnz": docs.nnz, "queries_nnz": qs.nnz},
              open(os.path.join(HERE, "workload_digests.json"), "w"), indent=1)
    ids, sc = oracle.topk_f64(docs, qs, 100)
    ids8, sc8 = oracle.topk_i64(docs, qs, 100)
    json.dump({"workload": w.name, "k": 100,
               "f64_ids": ids.tolist(), "f64_scores_hex": [[float(x).hex() for x in r] for r in sc],
               "i64_ids": ids8.tolist(), "i64_scores": sc8.tolist()},
              open(os.path.join(HERE, "tiny10k_oracle.json"), "w"))


if __name__ == "__main__":
    main()
