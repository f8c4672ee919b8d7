"""Convergence-window termination (Sec. IV-A) on the GPU: the run stops after
the same generation as the oracle's, in one call or many, alone, in a batch
and in the server, with the state bit-identical at the stop."""
import numpy as np
import pytest

import workloads
from gpu_common import assert_state_equal, say
from test_gpu_batch import View

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


@pytest.mark.parametrize("window,pieces", [(20, [5000]), (5, [3, 7, 100, 5000]), (32, [64] * 80),
                                           (2, [1] * 50)])
def test_single_instance_stops_with_the_oracle(qieo, oracle_mod, window, pieces):
    inst = workloads.small_instance()
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_convergence(window)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    total = sum(pieces)
    n = o.run_until_converged(total, window)
    say("window %d: oracle stops after %d generations" % (window, n))
    for p in pieces:
        g.step(p)
    conv, at = g.converged()
    assert g.generations == o.t == n
    assert conv == o.converged(window)
    if conv:
        assert at == n - 1
    assert_state_equal(g, o, label="window %d" % window)
    g.step(10)                                   # nothing runs after convergence
    assert g.generations == n


def test_window_must_be_set_first(qieo):
    inst = workloads.random_instance(50, 4, seed=1)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.step(1)
    with pytest.raises(qieo.QieoError) as ei:
        g.set_convergence(10)
    assert ei.value.code == qieo.QIEO_ESTATE
    with pytest.raises(qieo.QieoError):
        qieo.Instance(inst.values, inst.weights, inst.capacity, 4, 1).set_convergence(33)


def test_batch_members_stop_independently(qieo, oracle_mod):
    insts = [workloads.random_instance(ng, n_pop, seed=300 + k)
             for k, (ng, n_pop) in enumerate([(40, 8), (100, 16), (300, 4), (64, 32), (900, 7),
                                              (33, 2)])]
    b = qieo.Batch([(i.values, i.weights, i.capacity, i.n_pop, i.seed) for i in insts])
    b.set_convergence(6)
    for _ in range(4):
        b.step(150)
    for k, i in enumerate(insts):
        o = oracle_mod.Oracle(i.values, i.weights, i.capacity, i.n_pop, i.seed)
        n = o.run_until_converged(600, 6)
        assert b.generations(k) == n, (k, b.generations(k), n)
        assert b.converged(k)[0] == o.converged(6)
        assert_state_equal(View(b, k), o, label="batch conv %d" % k)


def test_server_retires_converged_requests(qieo, oracle_mod):
    reqs = [(workloads.random_instance(ng, n_pop, seed=500 + k), cap)
            for k, (ng, n_pop, cap) in enumerate([(60, 8, 2000), (120, 16, 40), (250, 4, 3000),
                                                  (80, 32, 2500)])]
    s = qieo.Server(1 << 28, gens_per_iter=13, convergence_window=8)
    tickets = [s.submit(i.values, i.weights, i.capacity, i.n_pop, i.seed, cap) for i, cap in reqs]
    for (i, cap), t in zip(reqs, tickets):
        res, _ = s.wait(t)
        o = oracle_mod.Oracle(i.values, i.weights, i.capacity, i.n_pop, i.seed)
        o.run_until_converged(cap, 8)
        ob = o.best()
        assert (res.fitness, res.generation, res.chromosome) == (ob.fitness, ob.generation,
                                                                  ob.chromosome)
        assert np.array_equal(res.alleles(i.n_items), ob.bits)
    s.close()
