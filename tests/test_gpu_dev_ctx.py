"""A caller's allocator and stream (qieo_dev_ctx) for single instances,
batches and the server: PyTorch's caching allocator and a PyTorch stream
give the same results as the library's defaults, every block the library
took is given back, and an allocator that fails after N blocks makes the
create call (or, for the server, the requests whose tables cannot be
allocated) fail with QIEO_ENOMEM without leaking what it had taken."""
import threading

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


class TorchAlloc:
    """Device blocks from PyTorch's caching allocator on one stream, counted;
    fail_after = N makes every request after the first N return NULL."""

    def __init__(self, stream, fail_after=None):
        import torch
        self.torch, self.stream = torch, stream
        self.fail_after = fail_after
        self.calls = 0
        self.live = {}
        self.lock = threading.Lock()

    def alloc(self, n):
        with self.lock:
            self.calls += 1
            if self.fail_after is not None and self.calls > self.fail_after:
                return 0
        p = self.torch.cuda.caching_allocator_alloc(n, device=0, stream=self.stream)
        with self.lock:
            self.live[p] = n
        return p

    def free(self, p):
        with self.lock:
            assert p in self.live, "free of a block the allocator did not hand out"
            del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


def _ctx(qieo, a, stream):
    return qieo.DeviceContext(a.alloc, a.free, stream.cuda_stream)


def _same_state(a, b, label):
    for key in ("alpha", "beta", "alleles", "fitness", "profit", "weight"):
        assert np.array_equal(a[key], b[key]), (label, key)
    assert a["elite"] == b["elite"], label


def test_instance_with_torch_allocator_and_stream(qieo):
    import torch
    inst = workloads.random_instance(3000, 40, seed=71)
    stream = torch.cuda.Stream()
    a = TorchAlloc(stream)
    for precision in (32, 64):
        ref = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                            precision=precision)
        g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=precision, ctx=_ctx(qieo, a, stream))
        assert a.live, "the caller's allocator was not used"
        for n in (1, 6, 6):                   # the repeated call is captured and replayed
            ref.step(n)
            g.step(n)
        if precision == 32:
            _same_state(ref.export_rows(), g.export_rows(), "binary32")
        else:
            x, y = ref.export_rows(amplitudes=False), g.export_rows(amplitudes=False)
            for key in ("alleles", "fitness"):
                assert np.array_equal(x[key], y[key]), key
        r1, r2 = ref.best(), g.best()
        assert (r1.fitness, r1.generation, r1.chromosome) == (r2.fitness, r2.generation,
                                                               r2.chromosome)
        assert np.array_equal(r1.bits, r2.bits)
        ref.close()
        g.close()
        assert not a.live, "blocks left after destroy: %s" % a.live
    say("  instance: %d blocks through the caller's allocator" % a.calls)


def test_instance_allocator_failing_after_n_blocks(qieo):
    import torch
    inst = workloads.random_instance(500, 8, seed=72)
    stream = torch.cuda.Stream()
    for n in (0, 1):                          # the arena, then the descriptor
        a = TorchAlloc(stream, fail_after=n)
        with pytest.raises(qieo.QieoError) as ei:
            qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          ctx=_ctx(qieo, a, stream))
        assert ei.value.code == qieo.QIEO_ENOMEM, ei.value
        assert not a.live, "failed create leaked %s" % a.live
    a = TorchAlloc(stream, fail_after=2)      # enough: the instance works
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      ctx=_ctx(qieo, a, stream))
    g.step(3)
    assert g.generations == 3
    g.close()
    assert not a.live


def _batch_problems():
    insts = [workloads.random_instance(ng, n_pop, seed=80 + k)
             for k, (ng, n_pop) in enumerate([(50, 32), (700, 64), (3000, 16), (9000, 128),
                                              (20000, 40), (130, 7)])]
    return [(i.values, i.weights, i.capacity, i.n_pop, i.seed) for i in insts]


def test_batch_with_torch_allocator_and_failures(qieo):
    import torch
    probs = _batch_problems()
    stream = torch.cuda.Stream()
    ref = qieo.Batch(probs)
    a = TorchAlloc(stream)
    b = qieo.Batch(probs, ctx=_ctx(qieo, a, stream))
    taken = a.calls
    for gens in ([3] * len(probs), [k % 4 for k in range(len(probs))], [5] * len(probs)):
        ref.step(gens)
        b.step(gens)
    for k in range(len(probs)):
        _same_state(ref.export_rows(k), b.export_rows(k), "member %d" % k)
    ref.close()
    b.close()
    assert not a.live, "batch left blocks: %s" % a.live
    say("  batch: %d blocks at create" % taken)
    # every prefix of the create's allocations fails cleanly
    for n in range(taken):
        f = TorchAlloc(stream, fail_after=n)
        with pytest.raises(qieo.QieoError) as ei:
            qieo.Batch(probs, ctx=_ctx(qieo, f, stream))
        assert ei.value.code == qieo.QIEO_ENOMEM, (n, ei.value)
        assert not f.live, "failed batch create (after %d blocks) leaked %s" % (n, f.live)


def test_server_with_torch_allocator_and_failures(qieo, oracle_mod):
    import torch
    reqs = [(workloads.random_instance(ng, n_pop, seed=90 + k), g)
            for k, (ng, n_pop, g) in enumerate([(300, 16, 7), (5000, 32, 11), (1200, 8, 30),
                                                (64, 3, 4)])]
    stream = torch.cuda.Stream()
    a = TorchAlloc(stream)
    s = qieo.Server(64 << 20, gens_per_iter=5, ctx=_ctx(qieo, a, stream))
    tickets = [s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, g) for i, g in reqs]
    results = [s.wait(t)[0] for t in tickets]
    s.close()
    assert not a.live, "server left blocks: %s" % a.live
    for (i, g), res in zip(reqs, results):
        o = oracle_mod.Oracle(i.values, i.weights, i.capacity, i.n_pop, i.seed)
        o.run(g)
        ob = o.best()
        assert (res.fitness, res.profit, res.weight, res.generation, res.chromosome) == \
            (ob.fitness, ob.profit, ob.weight, ob.generation, ob.chromosome)
        assert np.array_equal(res.alleles(i.n_items), ob.bits)
    say("  server: %d blocks through the caller's allocator" % a.calls)
    # the pool itself cannot be allocated: create fails
    f = TorchAlloc(stream, fail_after=0)
    with pytest.raises(qieo.QieoError) as ei:
        qieo.Server(64 << 20, ctx=_ctx(qieo, f, stream))
    assert ei.value.code == qieo.QIEO_ENOMEM and not f.live
    # the pool is there, the engine's tables are not: the request fails with
    # QIEO_ENOMEM and the server reports the error
    f = TorchAlloc(stream, fail_after=1)
    s = qieo.Server(64 << 20, ctx=_ctx(qieo, f, stream))
    i, g = reqs[0]
    t = s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, g)
    with pytest.raises(qieo.QieoError) as ei:
        s.wait(t)
    assert ei.value.code == qieo.QIEO_ENOMEM, ei.value
    assert s.stats()["error"] == qieo.QIEO_ENOMEM
    s.close()
    assert not f.live, "failed server leaked %s" % f.live
