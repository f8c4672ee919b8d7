"""Binary64 amplitudes (the paper's precision): bit-exact against the
oracle's binary64 variant, per generation and at the medium size."""
import os

import numpy as np
import pytest

import workloads
from gpu_common import assert_state_equal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


@pytest.mark.parametrize("ng,n_pop", [(100, 16), (257, 7), (4097, 5), (1500, 23)])
def test_f64_every_generation(qieo, oracle_mod, ng, n_pop):
    inst = workloads.random_instance(ng, n_pop, seed=ng + 64)
    say("f64 Ng=%d Np=%d" % (ng, n_pop))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=64)
    for gen in range(15):
        g.step(1)
        o.generation()
        assert_state_equal(g, o, label="f64 gen %d" % gen)
    g.step(40)
    o.run(40)
    assert_state_equal(g, o, label="f64 gen 55")


@pytest.mark.parametrize("tile,flags", [((1, 4), 0), ((2, 8), 3), ((4, 2), 1), ((4, 8), 6),
                                        ((2, 4), 7), ((2, 4), 16), ((2, 4), 18), ((2, 4), 22)])
def test_f64_work_shapes(qieo, oracle_mod, tile, flags):
    inst = workloads.random_instance(2000, 19, seed=6)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    g.set_tile(*tile)
    g.set_kernel_flags(flags)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=64)
    g.step(9)
    o.run(9)
    assert_state_equal(g, o, label="f64 tile %s" % (tile,))


def test_f64_medium_checkpoints(qieo, oracle_mod):
    inst = workloads.medium_instance()
    threads = min(16, os.cpu_count() or 1)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=threads, precision=64)
    done = 0
    for ck in (1, 10, 200):
        g.step(ck - done)
        o.run(ck - done)
        done = ck
        say("  f64 medium at generation %d" % ck)
        assert_state_equal(g, o, label="f64 medium gen %d" % ck)


def test_f64_rejects_f32_only_features(qieo):
    inst = workloads.random_instance(100, 4, seed=1)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    with pytest.raises(qieo.QieoError):
        g.set_pipeline(1)
    with pytest.raises(qieo.QieoError):
        g.set_persistent(2)


@pytest.mark.parametrize("ng,n_pop,flags", [(9000, 7, 22), (4097, 11, 18), (4096, 3, 22),
                                              (1025, 4, 22), (20000, 6, 22), (100, 5, 16),
                                              (3000, 5, 20), (9000, 7, 30), (1025, 3, 8)])
def test_f64_segment_order(qieo, oracle_mod, ng, n_pop, flags):
    """Binary64 amplitudes in segment order: several segments per row with a
    ragged last one, and rows shorter than one segment."""
    inst = workloads.random_instance(ng, n_pop, seed=ng + n_pop)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                      precision=64)
    g.set_kernel_flags(flags)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=64)
    for n in (1, 2, 5, 12):
        g.step(n)
        o.run(n)
        assert_state_equal(g, o, label="f64 segments t=%d" % o.t)
