"""Host logic of bench.py, checked on CPU: the multi-GPU refusal, the code digest that
keys committed traffic profiles, and the algorithmic-byte count of the roofline."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from workload import SparseRows  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_code_digest_ignores_comments_and_whitespace_only(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text('int f(int x) {  // one\n  return x + 1; /* two */ }\nconst char* s = "// kept";\n')
    b.write_text('int f(int x) {\n\n    return x + 1;  }  // other words\nconst char* s = "// kept";\n')
    c.write_text('int f(int x) {  // one\n  return x + 2; /* two */ }\nconst char* s = "// kept";\n')
    da, db, dc = (bench.code_digest([str(p)]) for p in (a, b, c))
    assert da == db and da != dc
    d = tmp_path / "d.hip"  # a comment marker inside a string literal is code
    d.write_text('int f(int x) {  // one\n  return x + 1; /* two */ }\nconst char* s = "// changed";\n')
    assert bench.code_digest([str(d)]) != da


def test_algorithmic_bytes_per_term_id_bytes():
    # two queries over a 4-term vocabulary: term 0 is in byte form (1 + 4/64 B per id),
    # the others take 2 B; 4 B weights; one 4 B score write per doc per query
    df = np.array([100, 10, 0, 7], dtype=np.int64)
    q = SparseRows(np.array([0, 2, 3], dtype=np.int64), np.array([0, 1, 3], dtype=np.int32),
                   np.ones(3, dtype=np.float32), 4)
    idb = np.array([1 + 4 / 64, 2, 2, 2])
    p_q, score, step = bench.algorithmic_bytes(df, q, 50, 4, idb)
    assert list(p_q) == [110, 7]
    assert score == round(100 * (1 + 4 / 64 + 4) + 10 * 6 + 7 * 6) + 2 * 50 * 4
    assert step == score + 2 * 50 * 4
    # a scalar id size and fused filtering (only written_docs scores written)
    _, score2, _ = bench.algorithmic_bytes(df, q, 50, 4, 2, written_docs=8)
    assert score2 == 117 * 6 + 2 * 8 * 4
