"""Block-max pruning (opts.prune): exact, so bit-identical to the search without it.

Pruning works in the non-seed tiles of fused candidate filtering (searches of 32+
queries): the query terms whose upper bounds sum below the seed bound's score are
non-essential, and a 64-posting block of such a term is skipped when no doc it can
hold can reach the bound. Candidates keep their complete sums, so the results must
equal the unpruned search bit for bit (fixed-point fp32, integer uint8), and the
oracle. The diagnostics count the blocks skipped.
"""
import numpy as np
import pytest

import workload
from helpers import csr
from parity_rules import check_batch

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


def _search(gs, torch, idx, qs, k, prune):
    b = idx.batch(qs, k, k_max=int(np.max(k)))
    opts = gs.make_opts("tiled", prune=prune)
    ids, sc = idx.search(b, idx.workspace(qs.n_rows, opts), opts)
    torch.cuda.synchronize()
    d = b.diagnostics()
    b.close()
    return ids.cpu().numpy(), sc.cpu().numpy(), d


@pytest.fixture(scope="module")
def skewed():
    # term 0: a tenth of the docs, weights up to 3; terms 1-5: half the docs, weights <= 0.02;
    # queries weigh term 0 heavily and terms 1-5 lightly, so terms 1-5 are non-essential and
    # their blocks over docs without term 0 can be skipped
    rng = np.random.default_rng(91)
    n, vocab = 300_000, 40  # 19 uint8 tiles of 16384 docs: enough for fused filtering
    rows = []
    for d in range(n):
        r = []
        if d % 10 == 3:
            r.append((0, float(rng.uniform(0.5, 3.0))))
        for t in range(1, 6):
            if rng.random() < 0.5:
                r.append((t, float(rng.uniform(0.001, 0.02))))
        for t in rng.choice(np.arange(6, vocab), size=int(rng.integers(0, 4)), replace=False):
            r.append((int(t), float(np.log1p(rng.lognormal(0, 0.8)))))
        rows.append(sorted(r))
    docs = csr(rows, vocab)
    qrows = []
    for i in range(40):
        q = [(0, float(rng.uniform(1.0, 3.0)))] + [(t, float(rng.uniform(0.01, 0.1))) for t in range(1, 6)]
        if i % 4 == 0:
            q += [(int(t), 0.2) for t in rng.choice(np.arange(6, vocab), size=3, replace=False)]
        qrows.append(sorted(q))
    return docs, csr(qrows, vocab)


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_pruning_is_exact_and_skips_blocks(skewed, precision):
    gs, torch = _gs()
    docs, qs = skewed
    idx = gs.Index.from_rows(docs, precision)
    k = np.full(qs.n_rows, 100, np.int32)
    a = _search(gs, torch, idx, qs, k, False)
    b = _search(gs, torch, idx, qs, k, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), "pruning changed the result"
    assert a[2][:, 6].sum() == 0 and b[2][:, 6].sum() > 0, "no block was skipped"
    check_batch(precision, docs, qs, b[0], b[1], k, what="pruned " + precision)


@pytest.mark.parametrize("precision", ["fp32", "u8"])
def test_pruning_on_the_synthetic_workload(precision):
    gs, torch = _gs()
    w = workload.WORKLOADS["mid-1m"]
    docs, qs = workload.make_collection(w), workload.make_queries(w, n=48)
    idx = gs.Index.from_rows(docs, precision)
    k = np.full(qs.n_rows, 1000, np.int32)
    a = _search(gs, torch, idx, qs, k, False)
    b = _search(gs, torch, idx, qs, k, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), "pruning changed the result"
    check_batch(precision, docs, qs.subset(np.arange(12)), b[0][:12], b[1][:12], k[:12], what="pruned 1M")


def test_pruning_needs_the_tiled_kernel_and_fp32_or_u8(skewed):
    gs, torch = _gs()
    docs, qs = skewed
    for precision, kernel in (("bf16", "tiled"), ("u8", "shared"), ("fp32", "group")):
        idx = gs.Index.from_rows(docs, precision)
        with pytest.raises(gs.GsError) as e:
            idx.search(idx.batch(qs, 10), idx.workspace(4), gs.make_opts(kernel, prune=True))
        assert e.value.code == gs.GS_EUNSUPPORTED
