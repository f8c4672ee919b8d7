"""qieo_best_noalloc (the best-so-far record without any allocation, for
callers that cannot allocate) against qieo_best, through the C ABI: two calls
in a row on instances of different sizes, the second smaller, each compared
word for word with qieo_best on the same handle; plus its argument checks."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


def _call(qieo, fn, h, n_words, fill, with_bits=True):
    """fn(h, &record, bits, n_words); with_bits False passes no bits buffer."""
    r = qieo.qieo_result()
    bits = np.full(max(n_words, 1), fill, dtype=np.uint32)
    ptr = bits.ctypes.data_as(ctypes.c_void_p) if with_bits else None
    rc = fn(h, ctypes.byref(r), ptr, n_words)
    return rc, r, bits[:n_words]


def _fields(r):
    return (r.fitness, r.profit, r.weight, r.feasible, r.generation, r.chromosome)


def test_best_noalloc_equals_best_on_two_calls_second_smaller(qieo):
    lib = qieo.lib
    for ng, n_pop, seed, gens in ((100_003, 7, 21, 9), (1000, 5, 22, 5)):
        inst = workloads.random_instance(ng, n_pop, seed=seed)
        g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
        g.step(gens)
        nw = (ng + 31) // 32
        rc1, r1, b1 = _call(qieo, lib.qieo_best, g.handle, nw, 0xDEADBEEF)
        rc2, r2, b2 = _call(qieo, lib.qieo_best_noalloc, g.handle, nw, 0x5A5A5A5A)
        assert rc1 == qieo.QIEO_OK and rc2 == qieo.QIEO_OK, qieo.qieo_last_error()
        assert _fields(r1) == _fields(r2) and r1.generation >= 0
        assert np.array_equal(b1, b2), "best bits differ (%d items)" % ng
        # the record alone (no bits), and a second call after the first
        rc3, r3, _ = _call(qieo, lib.qieo_best_noalloc, g.handle, 0, 0, with_bits=False)
        assert rc3 == qieo.QIEO_OK and _fields(r3) == _fields(r1)
        r4, b4 = qieo.qieo_best_noalloc(g.handle, ng)
        assert _fields(r4) == _fields(r1) and np.array_equal(b4, b1)
        say("  %d items: best %d (generation %d) equal through both entry points"
            % (ng, r1.fitness, r1.generation))
        g.close()


def test_best_noalloc_refuses_what_does_not_fit(qieo):
    lib = qieo.lib
    inst = workloads.random_instance(300, 3, seed=23)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.step(2)
    rc, _, _ = _call(qieo, lib.qieo_best_noalloc, g.handle, (300 + 31) // 32 - 1, 0)
    assert rc == qieo.QIEO_EINVAL                  # bits buffer too short
    rc = lib.qieo_best_noalloc(g.handle, None, None, 0)
    assert rc == qieo.QIEO_EINVAL                  # no output record
    g.close()
    ng = qieo.QIEO_BEST_NOALLOC_MAX_ITEMS + 1      # one item past the static staging
    v = np.ones(ng, np.int32)
    g = qieo.Instance(v, v, ng // 2, 1, 24)
    g.step(1)
    nw = (ng + 31) // 32
    rc, _, _ = _call(qieo, lib.qieo_best_noalloc, g.handle, nw, 0)
    assert rc == qieo.QIEO_EINVAL and "static staging" in qieo.qieo_last_error()
    # the record alone works at any size
    rc, r, _ = _call(qieo, lib.qieo_best_noalloc, g.handle, 0, 0, with_bits=False)
    rc2, r2, _ = _call(qieo, lib.qieo_best, g.handle, 0, 0, with_bits=False)
    assert rc == rc2 == qieo.QIEO_OK and _fields(r) == _fields(r2)
    g.close()
