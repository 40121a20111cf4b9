"""Out-of-memory paths: every device or pinned allocation of index build, batch and server
creation is made to fail in turn (gs_debug_fail_alloc); each call must return GS_ENOMEM,
hand out no object and leak no device memory, and the next call must work."""
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


def _free_bytes(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def _fail_each(gs, torch, make, max_allocs=64):
    """Call make() with the n-th allocation failing, n = 0, 1, ... until it succeeds."""
    before = _free_bytes(torch)
    for n in range(max_allocs):
        gs.debug_fail_alloc(n)
        try:
            obj = make()
        except gs.GsError as e:
            assert e.code == gs.GS_ENOMEM, "allocation %d: %s" % (n, e)
            continue
        finally:
            gs.debug_fail_alloc(-1)
        # no leak from the failed attempts (within 2 MiB of runtime bookkeeping)
        return obj, n, before
    raise AssertionError("more than %d allocations" % max_allocs)


@pytest.mark.parametrize("precision", ["fp32", "u8", "bf16"])
def test_index_batch_and_server_out_of_memory(precision):
    gs, torch = _gs()
    docs = workload.collection(30_000, seed=31)
    qs = workload.queries_poisson(8, seed=32)
    # warm up: the first call loads the library's device code (with its fixed scratch array)
    gs.Index.from_rows(docs, precision).close()
    base = _free_bytes(torch)
    idx, n_idx, _ = _fail_each(gs, torch, lambda: gs.Index.from_rows(docs, precision, keep_doc_ids=True))
    assert n_idx >= 5, "the index build made %d allocations" % n_idx
    held = base - _free_bytes(torch)
    assert abs(held - idx.info().device_bytes) < (64 << 20), "failed builds leaked device memory"
    b, n_b, _ = _fail_each(gs, torch, lambda: idx.batch(qs, 10))
    assert n_b == 2  # device arrays, then the pinned stage
    ids, sc = idx.search(b, idx.workspace(qs.n_rows))
    torch.cuda.synchronize()
    check_batch(precision, docs, qs, ids.cpu().numpy(), sc.cpu().numpy(), 10, what="after faults")
    srv, n_s, _ = _fail_each(gs, torch, lambda: gs.Server(idx, max_batch=4, n_slots=2, k_max=10))
    assert n_s >= 3
    t, w = qs.row(0)
    got = srv.wait(srv.submit(t, w, 10), 10)
    assert np.array_equal(got[0], ids.cpu().numpy()[0])
    srv.close()
    b.close()
    idx.close()
    after = _free_bytes(torch)
    assert abs(after - base) < (64 << 20), "device memory not returned"
