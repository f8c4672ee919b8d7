"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit for
bit (amplitudes as binary32 bit patterns, alleles, integer fitness, elite
index, best-so-far record), generation by generation."""
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


def _pair(qieo, oracle_mod, inst, threads=1, tile=None):
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    if tile is not None:
        g.set_tile(*tile)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=threads)
    return g, o


def test_initial_state(qieo, oracle_mod):
    inst = workloads.random_instance(300, 5, seed=1)
    g, o = _pair(qieo, oracle_mod, inst)
    st = g.export_rows()
    a, b = o.amplitudes()
    assert np.array_equal(st["alpha"], a) and np.array_equal(st["beta"], b)
    assert st["elite"] == -1
    r = g.best()
    assert r.generation == -1


def test_small_instance_every_generation(qieo, oracle_mod):
    """Ng=100, Np=16, 500 generations, seed 0: full state after every one."""
    inst = workloads.small_instance()
    say("small instance %s" % inst.name)
    g, o = _pair(qieo, oracle_mod, inst)
    for gen in range(inst.generations):
        g.step(1)
        o.generation()
        assert_state_equal(g, o, label="gen %d" % gen)
    assert g.generations == inst.generations


# ragged sizes: genes per row around the 64-gene pitch and 256-gene chunk
# boundaries, single rows, odd row counts; every work shape
SHAPES = [
    (1, 1), (3, 1), (63, 2), (64, 3), (65, 4), (255, 5), (256, 6), (257, 7),
    (511, 3), (1000, 9), (4097, 5), (20000, 3), (130, 33),
]


@pytest.mark.parametrize("ng,n_pop", SHAPES)
def test_ragged_shapes_every_generation(qieo, oracle_mod, ng, n_pop):
    inst = workloads.random_instance(ng, n_pop, seed=ng * 7 + n_pop)
    say("ragged Ng=%d Np=%d" % (ng, n_pop))
    g, o = _pair(qieo, oracle_mod, inst)
    for gen in range(12):
        g.step(1)
        o.generation()
        assert_state_equal(g, o, label="Ng=%d Np=%d gen %d" % (ng, n_pop, gen))


@pytest.mark.parametrize("tile,flags", [((1, 1), 0), ((1, 3), 1), ((2, 2), 2), ((2, 16), 3),
                                        ((4, 1), 1), ((4, 5), 3), ((4, 16), 0), ((1, 8), 3),
                                        ((1, 2), 4), ((2, 4), 8), ((4, 8), 15), ((4, 3), 12),
                                        ((2, 8), 11), ((1, 16), 9)])
def test_work_shapes_same_trajectory(qieo, oracle_mod, tile, flags):
    inst = workloads.random_instance(1500, 23, seed=99)
    say("tile %s flags %d" % (tile, flags))
    g, o = _pair(qieo, oracle_mod, inst, tile=tile)
    g.set_kernel_flags(flags)
    assert g.tile() == tile
    for step in (1, 2, 7):
        g.step(step)
        o.run(step)
        assert_state_equal(g, o, label="tile %s t=%d" % (tile, o.t))


def test_split_steps_equal_one_step(qieo, oracle_mod):
    inst = workloads.random_instance(777, 19, seed=4)
    a = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    b = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    a.step(30)
    for n in (1, 4, 0, 10, 15):
        b.step(n)
    sa, sb = a.export_rows(), b.export_rows()
    for k in ("alpha", "beta", "alleles", "fitness", "profit", "weight"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["elite"] == sb["elite"]
    assert a.best() .__dict__.keys() == b.best().__dict__.keys()
    ra, rb = a.best(), b.best()
    assert (ra.fitness, ra.generation, ra.chromosome) == (rb.fitness, rb.generation, rb.chromosome)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(30)
    assert_state_equal(b, o, label="split")


def test_async_steps(qieo, oracle_mod):
    inst = workloads.random_instance(2000, 40, seed=8)
    g, o = _pair(qieo, oracle_mod, inst)
    for _ in range(5):
        g.step_async(3)
    g.sync()
    o.run(15)
    assert_state_equal(g, o, label="async")


def test_medium_instance_checkpoints(qieo, oracle_mod):
    """Ng=10,000, Np=1024, 1000 generations, seed 1: full state at several
    generations and at the end (oracle row-threaded)."""
    inst = workloads.medium_instance()
    threads = min(16, os.cpu_count() or 1)
    say("medium instance, oracle threads %d" % threads)
    g, o = _pair(qieo, oracle_mod, inst, threads=threads)
    done = 0
    for ck in (1, 2, 10, 100, 400, 1000):
        g.step(ck - done)
        o.run(ck - done)
        done = ck
        say("  compare at generation %d" % ck)
        assert_state_equal(g, o, label="medium gen %d" % ck)


@pytest.mark.parametrize("pipeline", [1, 2, 3, 4])
@pytest.mark.parametrize("ng,n_pop", [(100, 16), (1000, 9), (4097, 5), (300, 130)])
def test_unfused_pipelines_same_trajectory(qieo, oracle_mod, pipeline, ng, n_pop):
    """The four-launch pipelines (device, fused-into-Evaluation or host
    DetermineElite) follow the oracle bit for bit, also when the pipeline
    changes between calls."""
    inst = workloads.random_instance(ng, n_pop, seed=ng + pipeline)
    say("pipeline %d Ng=%d Np=%d" % (pipeline, ng, n_pop))
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_pipeline(pipeline)
    for step in (1, 1, 5):
        g.step(step)
        o.run(step)
        assert_state_equal(g, o, label="pipeline %d t=%d" % (pipeline, o.t))
    g.set_pipeline(0)
    g.step(3)
    g.set_pipeline(pipeline)
    g.step(4)
    o.run(7)
    assert_state_equal(g, o, label="pipeline %d mixed t=%d" % (pipeline, o.t))


def test_stage_timing(qieo):
    inst = workloads.random_instance(5000, 64, seed=3)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_timing(True)
    g.set_pipeline(1)
    g.step(4)
    st = g.stage_time(reset=True)
    assert st["cip"][0] == st["qip"][0] == st["fe"][0] == st["de"][0] == 4
    assert all(st[k][1] > 0 for k in ("cip", "qip", "fe", "de"))
    g.set_pipeline(3)
    g.step(2)
    st = g.stage_time()
    assert st["de"][0] == 2 and st["de"][1] > 0


def test_autotuner_picks_a_shape_used_by_create(qieo, oracle_mod, tmp_path):
    qieo.qieo_tune_db_clear()
    r = qieo.qieo_autotune(3000, 48, trial_generations=2)
    say("autotune 48 x 3000: %s" % r)
    assert r["candidates"] > 10
    assert r["ms_per_generation"] <= r["worst_ms_per_generation"]
    inst = workloads.random_instance(3000, 48, seed=77)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    assert g.tile() == (r["rows_per_block"], r["waves_per_block"])
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.step(6)
    o.run(6)
    assert_state_equal(g, o, label="tuned shape")
    path = str(tmp_path / "tune.json")
    qieo.qieo_tune_db_save(path)
    qieo.qieo_tune_db_clear()
    assert qieo.qieo_tune_db_load(path) == 1
    qieo.qieo_tune_db_clear()


@pytest.mark.parametrize("ng,n_pop", [(100, 16), (700, 37), (3000, 20), (64, 1024), (257, 3),
                                      (500, 24), (1, 1), (2000, 9)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_persistent_path_same_trajectory(qieo, oracle_mod, ng, n_pop, mode):
    """Per-generation launches (mode 0), the LDS-resident single-workgroup
    loop where the state fits LDS (mode 1, else per-generation launches) and
    the global-memory single-workgroup loop where it does not (mode 2) all
    follow the oracle, and switching between them between calls is seamless."""
    inst = workloads.random_instance(ng, n_pop, seed=ng * 3 + n_pop)
    say("persistent mode %d Ng=%d Np=%d" % (mode, ng, n_pop))
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_persistent(mode)
    for step in (1, 7, 30):
        g.step(step)
        o.run(step)
        assert_state_equal(g, o, label="persistent %d t=%d" % (mode, o.t))
    for other in (mode + 1) % 3, (mode + 2) % 3:
        g.set_persistent(other)
        g.step(5)
        o.run(5)
        assert_state_equal(g, o, label="persistent %d -> %d t=%d" % (mode, other, o.t))


@pytest.mark.parametrize("graph", [0, 1])
def test_graph_replay_same_trajectory(qieo, oracle_mod, graph):
    """Captured-graph replay of whole calls (a call is captured when it
    repeats: same n three times, another n, a shape change) follows the
    oracle."""
    inst = workloads.random_instance(6000, 40, seed=12)
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_persistent(0)
    g.set_graph(graph)
    for n, tile in ((5, None), (5, None), (5, None), (3, None), (3, None), (5, (2, 4)),
                    (5, (2, 4)), (5, (2, 4))):
        if tile:
            g.set_tile(*tile)
        g.step(n)
        o.run(n)
        assert_state_equal(g, o, label="graph %d t=%d" % (graph, o.t))


def test_graph_capture_with_concurrent_device_calls(qieo, oracle_mod):
    """A call whose graph capture overlaps another thread's allocations,
    frees and copies (a server or a second instance) still runs every
    generation once: the capture either completes or the same launches are
    enqueued directly."""
    import threading
    inst = workloads.random_instance(3000, 24, seed=14)
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_persistent(0)
    g.set_graph(1)
    stop = threading.Event()
    errors = []

    def churn():
        other = workloads.random_instance(500, 8, seed=15)
        try:
            while not stop.is_set():
                h = qieo.Instance(other.values, other.weights, other.capacity, other.n_pop,
                                  other.seed)
                h.step(1)
                h.best()
                h.close()
        except Exception as exc:            # reported by the main thread
            errors.append(exc)

    th = threading.Thread(target=churn)
    th.start()
    try:
        for n in (2, 2, 3, 3, 4, 4, 7, 7, 9, 9, 9):    # a new capture on every repeat
            g.step(n)
            o.run(n)
            assert_state_equal(g, o, label="concurrent capture t=%d" % o.t)
    finally:
        stop.set()
        th.join()
    assert not errors, errors


@pytest.mark.parametrize("ng,n_pop", [(1, 3), (255, 7), (1024, 3), (1025, 2), (2048, 4),
                                      (4096, 5), (4097, 9), (9000, 33), (20000, 12)])
@pytest.mark.parametrize("flags", [16, 22, 31])
def test_segment_order_same_trajectory(qieo, oracle_mod, ng, n_pop, flags):
    """The segment-order generation (one workgroup per 1024-gene segment of a
    row, then a launch closing the rows) follows the oracle on rows shorter
    than one segment, exactly one or two, and several with a ragged last one;
    direct launches and graph replay."""
    inst = workloads.random_instance(ng, n_pop, seed=ng + 31 * n_pop)
    say("segments flags %d Ng=%d Np=%d" % (flags, ng, n_pop))
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_persistent(0)
    g.set_kernel_flags(flags)
    assert g.kernel_flags() == flags
    for n in (1, 2, 3, 3, 3, 9):
        g.step(n)
        o.run(n)
        assert_state_equal(g, o, label="segments %d t=%d" % (flags, o.t))


def test_segment_order_with_convergence_window(qieo, oracle_mod):
    inst = workloads.small_instance()
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_persistent(0)
    g.set_kernel_flags(22)
    g.set_convergence(20)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    n = o.run_until_converged(5000, 20)
    for p in (7, 100, 5000):
        g.step(p)
    conv, at = g.converged()
    assert conv and at == n - 1 and g.generations == n
    assert_state_equal(g, o, label="segments converged")
