"""The C-ABI library loads on a machine without a GPU and exports every symbol the header declares (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpusparse.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(gs_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("gs_build_index", "gs_search", "gs_search_batch", "gs_batch_create", "gs_free_index",
                 "gs_workspace_size", "gs_index_info", "gs_layout_host", "gs_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2606_26441_amd as gs
    lib = ctypes.CDLL(gs.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_status_strings_and_version_without_gpu():
    import paper_2606_26441_amd as gs
    assert "gfx950" in gs.version()
    for code in gs._STATUS:
        assert gs.lib.gs_status_string(code).decode() != "unknown status"
    assert gs.lib.gs_status_string(-99).decode() == "unknown status"


@pytest.mark.parametrize("case", ["term_range", "negative_weight", "nan_weight", "duplicate", "row_ptr"])
def test_build_index_rejects_bad_input_before_touching_the_device(case):
    import paper_2606_26441_amd as gs
    rp = np.array([0, 2, 3], np.int64)
    t = np.array([1, 4, 2], np.int32)
    w = np.array([0.5, 1.0, 2.0], np.float32)
    if case == "term_range":
        t[1] = 10
    elif case == "negative_weight":
        w[0] = -1.0
    elif case == "nan_weight":
        w[2] = np.nan
    elif case == "duplicate":
        t[1] = 1
    elif case == "row_ptr":
        rp[1] = 4
    with pytest.raises(gs.GsError) as e:
        gs.layout_host(rp, t, w, vocab=10)
    assert e.value.code == gs.GS_EINVAL
    h = ctypes.c_void_p()
    rc = gs.lib.gs_build_index(rp.ctypes.data, 2, t.ctypes.data, w.ctypes.data, 3, 10, 0, 0, None, ctypes.byref(h))
    assert rc == gs.GS_EINVAL and not h.value
    assert gs.lib.gs_last_error().decode() != ""


def test_unknown_precision_and_flags_are_rejected():
    import paper_2606_26441_amd as gs
    rp = np.array([0, 1], np.int64)
    t = np.array([1], np.int32)
    w = np.array([0.5], np.float32)
    h = ctypes.c_void_p()
    assert gs.lib.gs_build_index(rp.ctypes.data, 1, t.ctypes.data, w.ctypes.data, 1, 4, 7, 0, None,
                                 ctypes.byref(h)) == gs.GS_EINVAL
    assert gs.lib.gs_build_index(rp.ctypes.data, 1, t.ctypes.data, w.ctypes.data, 1, 4, 0, 8, None,
                                 ctypes.byref(h)) == gs.GS_EINVAL
