"""The allocation-free search (gs_search_batch_noalloc) against gs_search_batch.

Through the C ABI: the same batch searched with a caller workspace and with the
library's fixed scratch array must give identical ids and scores (the fp32
fixed-point, bf16 fp64-rescored and uint8 sums do not depend on the query
tiling), on two calls in a row, the second with fewer queries, so the second
call runs on scratch that still holds the first call's contents.
"""
import numpy as np
import pytest

import workload
from parity_rules import check_batch

pytestmark = pytest.mark.gpu


def _gs():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2606_26441_amd as gs
    return gs, torch


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
@pytest.mark.parametrize("kernel", ["tiled", "shared", "group"])
def test_noalloc_matches_the_workspace_search(precision, kernel):
    gs, torch = _gs()
    docs = workload.collection(150_000, seed=81)
    qs = workload.queries_lognormal(40, seed=82)
    ks = workload.k_mix(qs.n_rows, seed=83)
    idx = gs.Index.from_rows(docs, precision)
    opts = gs.make_opts(kernel)
    batch = gs.Batch.reserve(idx, qs.n_rows, qs.nnz, 1000)
    dt = gs.SCORE_DTYPES[idx.precision]
    for n in (qs.n_rows, 9):  # the second call: fewer queries, on the first call's leftovers
        sub, kk = qs.subset(np.arange(n)), ks[:n]
        batch.update(sub, kk)
        ref = idx.search(batch, idx.workspace(qs.n_rows, opts), opts)
        ids = torch.full((qs.n_rows, 1000), -7, dtype=torch.int32, device="cuda")
        sc = torch.zeros((qs.n_rows, 1000), dtype=dt, device="cuda")
        idx.search_noalloc(batch, (ids, sc), opts)
        torch.cuda.synchronize()
        r_ids, r_sc = ref[0].cpu().numpy(), ref[1].cpu().numpy()
        g_ids, g_sc = ids.cpu().numpy(), sc.cpu().numpy()
        assert np.array_equal(g_ids, r_ids), "ids differ (%d queries)" % n
        assert np.array_equal(g_sc.view(np.uint8), r_sc.view(np.uint8)), "scores differ (%d queries)" % n
        check_batch(precision, docs, sub, g_ids[:n], g_sc[:n], kk, what="noalloc %s %d" % (precision, n))
    batch.close()
    idx.close()
