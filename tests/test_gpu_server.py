"""The continuous-batching server: results of requests that share the GPU
(admitted and retired at different iterations, under a memory budget that
forces queueing) equal, bit for bit, what the oracle computes for each
request alone."""
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


def footprint(ng, n_pop):
    """Device bytes of one population (upper estimate of the library's arena)."""
    pitch = (ng + 63) // 64 * 64
    nchunk = (pitch + 255) // 256
    return 2 * (n_pop * pitch + 256) * 4 + 2 * n_pop * nchunk * 32 + 2 * nchunk * 1024 + \
        6 * n_pop * 4 + nchunk * 32 + 16 * 256


def _requests(n, seed0):
    rng = np.random.default_rng(seed0)
    out = []
    for k in range(n):
        ng = int(rng.integers(20, 3000))
        n_pop = int(rng.choice([1, 7, 16, 40, 64]))
        gens = int(rng.integers(1, 60))
        out.append((workloads.random_instance(ng, n_pop, seed=seed0 + k), gens))
    return out


def _check_against_oracle(oracle_mod, inst, gens, res):
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(gens)
    ob = o.best()
    assert (res.fitness, res.profit, res.weight, res.generation, res.chromosome) == \
        (ob.fitness, ob.profit, ob.weight, ob.generation, ob.chromosome)
    assert np.array_equal(res.alleles(inst.n_items), ob.bits)


@pytest.mark.parametrize("onchip", [True, False])
def test_server_continuous_batching_matches_oracle(qieo, oracle_mod, onchip):
    """With the residents in batched on-chip launches (the default) and in
    per-generation launches only."""
    reqs = _requests(24, 5000)
    sizes = sorted(footprint(i.n_items, i.n_pop) for i, _ in reqs)
    budget = sizes[-1] + sizes[-2] + sizes[-3]          # room for about three at a time
    say("server budget %d bytes for %d requests, on-chip %s" % (budget, len(reqs), onchip))
    s = qieo.Server(budget, max_resident=0, gens_per_iter=7)
    s.set_onchip(onchip)
    tickets = [s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, g) for i, g in reqs]
    results = [s.wait(t) for t in tickets]
    st = s.stats()
    say("  stats %s" % st)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_resident"] >= 2                     # requests overlapped on the GPU
    assert st["peak_pool_used"] <= budget
    assert st["iterations"] > 3
    for (inst, g), (res, lat) in zip(reqs, results):
        assert lat > 0
        _check_against_oracle(oracle_mod, inst, g, res)
    s.close()


def test_server_resident_cap_and_alone_equivalence(qieo):
    reqs = _requests(10, 7000)
    s = qieo.Server(1 << 30, max_resident=2, gens_per_iter=5)
    tickets = [s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, g) for i, g in reqs]
    for (inst, g), t in zip(reqs, tickets):
        res, _ = s.wait(t)
        alone = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
        alone.step(g)
        ra = alone.best()
        assert (res.fitness, res.generation, res.chromosome) == (ra.fitness, ra.generation,
                                                                  ra.chromosome)
        assert np.array_equal(res.bits, ra.bits)
    assert s.stats()["peak_resident"] <= 2
    s.close()


def test_server_rejects_population_larger_than_budget(qieo):
    s = qieo.Server(1 << 20, gens_per_iter=4)
    big = workloads.random_instance(5000, 64, seed=3)            # ~2.6 MB of amplitudes
    small = workloads.random_instance(100, 4, seed=4)
    t_big = s.submit(big.values, big.weights, big.capacity, big.n_pop, big.seed, 3)
    t_small = s.submit(small.values, small.weights, small.capacity, small.n_pop, small.seed, 3)
    with pytest.raises(qieo.QieoError) as ei:
        s.wait(t_big)
    assert ei.value.code == qieo.QIEO_ENOMEM
    res, _ = s.wait(t_small)
    assert res.generation >= 0
    s.close()


def test_server_concurrent_submitters(qieo, oracle_mod):
    reqs = _requests(16, 9000)
    s = qieo.Server(1 << 28, gens_per_iter=9)
    tickets = [None] * len(reqs)

    def submitter(lo):
        for k in range(lo, len(reqs), 4):
            i, g = reqs[k]
            tickets[k] = s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, g)

    th = [threading.Thread(target=submitter, args=(lo,)) for lo in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert len(set(tickets)) == len(reqs)
    for (inst, g), t in zip(reqs, tickets):
        res, _ = s.wait(t)
        _check_against_oracle(oracle_mod, inst, g, res)
        s.release(t)
    s.close()
