"""Parity at the full size of the largest single-instance workload
(Np = 4096, Ng = 200,000, seed 2) in the launch configuration the benchmark
times: every chromosome's fitness, the elite and the best-so-far record bit
for bit at early generations (row-threaded oracle over the whole population),
amplitudes and alleles of sampled rows, then invariants at generation 200;
the same early checks with binary64 amplitudes."""
import os

import numpy as np
import pytest

import workloads
from gpu_common import assert_state_equal, bits_equal, say

pytestmark = pytest.mark.gpu

SAMPLE_ROWS = [0, 1, 2, 3, 1000, 2047, 2048, 3333, 4092, 4093, 4094, 4095]


@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


def test_large_instance_full_size(qieo, oracle_mod):
    inst = workloads.large_instance()
    threads = min(16, os.cpu_count() or 1)
    say("large instance %s, oracle threads %d" % (inst.name, threads))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    say("  work shape %s" % (g.tile(),))
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=threads)
    done = 0
    for ck in (1, 2, 3, 5):
        g.step(ck - done)
        o.run(ck - done)
        done = ck
        say("  compare at generation %d" % ck)
        # all rows: fitness, profit, weight (no amplitudes)
        st = g.export_rows(0, inst.n_pop, amplitudes=False, alleles=False)
        f_o, P_o, W_o = o.fitness()
        assert np.array_equal(st["fitness"].astype(np.int64), f_o)
        assert np.array_equal(st["profit"].astype(np.int64), P_o)
        assert np.array_equal(st["weight"].astype(np.int64), W_o)
        assert st["elite"] == o.elite
        # sampled rows: amplitudes and alleles, plus the elite's row
        rows = sorted(set(SAMPLE_ROWS + [o.elite]))
        assert_state_equal(g, o, rows=rows, label="large gen %d" % ck)
    del o

    say("  run to generation %d" % inst.generations)
    g.step(inst.generations - done)
    assert g.generations == inst.generations
    st = g.export_rows(0, inst.n_pop, amplitudes=False, alleles=False)
    fit = st["fitness"].astype(np.int64)
    assert st["elite"] == int(np.argmax(fit))            # lowest index among ties
    v = inst.values.astype(np.int64)
    w = inst.weights.astype(np.int64)
    for r in SAMPLE_ROWS:
        s = g.export_rows(r, 1)
        x = s["alleles"][0].astype(np.int64)
        P, W = int(x @ v), int(x @ w)
        assert (s["profit"][0], s["weight"][0]) == (P, W)
        assert s["fitness"][0] == (P if W <= inst.capacity else -(W - inst.capacity))
        a = s["alpha"][0].astype(np.float64)
        b = s["beta"][0].astype(np.float64)
        assert np.abs(a * a + b * b - 1.0).max() <= 1e-5
    best = g.best()
    bits = best.alleles(inst.n_items).astype(np.int64)
    assert int(bits @ v) == best.profit and int(bits @ w) == best.weight
    assert best.feasible and best.fitness == best.profit
    assert best.fitness >= int(fit.max())
    lp = oracle_mod.knap_lp_bound(inst.values, inst.weights, inst.capacity)
    assert best.fitness <= lp
    say("  best %d (generation %d), LP bound %.0f" % (best.fitness, best.generation, lp))


def test_large_instance_binary64(qieo, oracle_mod):
    inst = workloads.large_instance()
    threads = min(16, os.cpu_count() or 1)
    say("large instance %s, binary64, oracle threads %d" % (inst.name, threads))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    say("  variant bits %d" % g.kernel_flags())
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=threads, precision=64)
    done = 0
    for ck in (1, 2, 4):
        g.step(ck - done)
        o.run(ck - done)
        done = ck
        say("  compare at generation %d" % ck)
        st = g.export_rows(0, inst.n_pop, amplitudes=False, alleles=False)
        f_o, P_o, W_o = o.fitness()
        assert np.array_equal(st["fitness"].astype(np.int64), f_o)
        assert np.array_equal(st["profit"].astype(np.int64), P_o)
        assert np.array_equal(st["weight"].astype(np.int64), W_o)
        assert st["elite"] == o.elite
        rows = sorted(set(SAMPLE_ROWS + [o.elite]))
        assert_state_equal(g, o, rows=rows, label="large f64 gen %d" % ck)
