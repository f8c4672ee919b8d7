"""The C-ABI library loads without a GPU, exports every symbol its header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(qieo_[a-z_0-9]+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for core in ("qieo_create", "qieo_step", "qieo_best", "qieo_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2609_30862_amd import qieo
    lib = ctypes.CDLL(qieo.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_version():
    from paper_2609_30862_amd import qieo
    assert "gfx950" in qieo.qieo_version()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert qieo.lib.qieo_strerror(code)


@pytest.mark.parametrize("values,weights,cap,n_pop,code", [
    ([1, -2], [3, 4], 3, 4, -1),           # negative value
    ([1, 2], [3, -4], 3, 4, -1),           # negative weight
    ([1, 2], [3, 4], -1, 4, -1),           # negative capacity
    ([1, 2], [3, 4], 3, 0, -1),            # empty population
    ([2**31 - 1, 1], [3, 4], 3, 4, -2),    # profit sum overflows int32
    ([1, 1], [2**31 - 1, 4], 3, 4, -2),    # weight sum overflows int32
])
def test_create_validates_before_device(values, weights, cap, n_pop, code):
    from paper_2609_30862_amd import qieo
    with pytest.raises(qieo.QieoError) as ei:
        qieo.Instance(values, weights, cap, n_pop, 0)
    assert ei.value.code == code


def test_create_rejects_empty_items():
    from paper_2609_30862_amd import qieo
    h = ctypes.c_void_p()
    items = np.zeros((1, 2), np.int32)
    rc = qieo.lib.qieo_create(items.ctypes.data_as(ctypes.c_void_p), 0, 1, 1, 0,
                              ctypes.byref(h))
    assert rc == qieo.QIEO_EINVAL and not h.value
    rc = qieo.lib.qieo_create(None, 3, 1, 1, 0, ctypes.byref(h))
    assert rc == qieo.QIEO_EINVAL


def test_null_handles_are_rejected():
    from paper_2609_30862_amd import qieo
    L = qieo.lib
    assert L.qieo_step(None, 1) == qieo.QIEO_EINVAL
    assert L.qieo_sync(None) == qieo.QIEO_EINVAL
    assert L.qieo_set_tile(None, 1, 1) == qieo.QIEO_EINVAL
    n = ctypes.c_size_t(0)
    assert L.qieo_state_size(None, ctypes.byref(n)) == qieo.QIEO_EINVAL
    buf = np.zeros(64, np.uint8)
    assert L.qieo_export_state(None, buf.ctypes.data_as(ctypes.c_void_p), 64) == qieo.QIEO_EINVAL
    assert L.qieo_import_state(None, buf.ctypes.data_as(ctypes.c_void_p), 64) == qieo.QIEO_EINVAL
    assert L.qieo_set_persistent(None, 1) == qieo.QIEO_EINVAL
    assert L.qieo_set_kernel_flags(None, 0) == qieo.QIEO_EINVAL
    assert L.qieo_batch_set_segment_order(None, 1) == qieo.QIEO_EINVAL
    assert L.qieo_batch_set_onchip(None, 1) == qieo.QIEO_EINVAL
    assert L.qieo_server_set_onchip(None, 1) == qieo.QIEO_EINVAL
    assert L.qieo_batch_set_barrier_timeout(None, 1) == qieo.QIEO_EINVAL
    n32 = ctypes.c_int32(0)
    assert L.qieo_batch_onchip_launches(None, ctypes.byref(n32)) == qieo.QIEO_EINVAL
    L.qieo_destroy(None)



@pytest.mark.parametrize("n_items,n_pop", [
    ((1 << 30) - 256, 65),     # just over 2^36 genes
    (64, 2**31 - 1),           # short rows, the largest population
    (1, (1 << 30) + 1),        # rows padded to 64 genes count as 64
])
def test_create_rejects_populations_beyond_2_36_genes(n_items, n_pop):
    # the size check comes before the item table is read, so a short table
    # stands in for a long one here
    from paper_2609_30862_amd import qieo
    items = np.zeros((4, 2), np.int32)
    h = ctypes.c_void_p()
    rc = qieo.lib.qieo_create(items.ctypes.data_as(ctypes.c_void_p), n_items, 1, n_pop, 0,
                              ctypes.byref(h))
    assert rc == qieo.QIEO_EINVAL and not h.value
    assert b"2^36" in qieo.lib.qieo_last_error()


@pytest.mark.parametrize("n_items,n_pop,trials", [
    (2**31 - 1, 1, 2),         # beyond 2^30 - 256 items
    ((1 << 30) - 256, 65, 2),  # beyond 2^36 genes
    (100, 0, 2),               # empty population
    (100, 4, 0),               # no trial generations
    (100, 4, 1001),            # too many trial generations
])
def test_autotune_rejects_bad_shapes_before_allocating(n_items, n_pop, trials):
    # items NULL would otherwise size a synthetic table of n_items entries
    from paper_2609_30862_amd import qieo
    rc = qieo.lib.qieo_autotune(n_items, n_pop, None, 0, trials, None)
    assert rc == qieo.QIEO_EINVAL
