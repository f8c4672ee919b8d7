"""The on-chip grid loop (qieo_set_persistent mode 3, and mode 1's choice for
calls of >= 4 generations): one cooperative launch per call, amplitudes in
registers, a grid barrier per generation.  Against the oracle at the medium
workload and on shapes that exercise its item split (rows per workgroup,
items per wave, waves whose items span rows, waves with no item, rows
shorter than a chunk, a ragged last workgroup), across calls that mix it
with per-generation launches, exports and checkpoints, and with a
convergence window."""
import os

import numpy as np
import pytest

import workloads
from gpu_common import assert_state_equal, say

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


def _pair(qieo, oracle_mod, inst, mode=3):
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_persistent(mode)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=THREADS)
    return g, o


def _step_path(g, n):
    """Steps n generations; returns the path the call took and the number of
    launches the library timed for it (one for a whole-call launch)."""
    g.set_timing(True)
    g.kernel_time(reset=True)
    g.step(n)
    launches, _ = g.kernel_time(reset=True)
    g.set_timing(False)
    return g.call_path(), launches


def test_medium_workload_every_call_length(qieo, oracle_mod):
    """1024 x 10,000 (seed 1): calls of 1, 2, 7 and 40 generations, the
    whole state against the oracle after each; every call is one launch."""
    inst = workloads.medium_instance()
    g, o = _pair(qieo, oracle_mod, inst)
    for n in (1, 2, 7, 40):
        assert _step_path(g, n) == (qieo.PATH_ONCHIP, 1), "call of %d generations" % n
        o.run(n)
        assert_state_equal(g, o, label="medium after %d generations" % o.t)
        say("  medium: %d generations equal the oracle" % o.t)
    g.close()


@pytest.mark.parametrize("ng,n_pop,wmax", [
    (3000, 1000, 10),     # 12 chunks, 4 rows per workgroup, last workgroup ragged
    (700, 2000, 10),      # 3 chunks: a wave's items span rows
    (60, 4000, 10),       # one 64-gene chunk per row, 16 rows per workgroup
    (9000, 300, 10),      # 2 rows per workgroup, 36 chunks
    (12000, 50, 10),      # fewer rows than compute units, 47 chunks a row
    (100, 5, 10),         # five workgroups of one item each
    # item values at the packed tables' limit (profits up to 2^14 - 1) and
    # beyond it (the variant with a table for each)
    (3000, 1000, 16378),
    (9000, 300, 30000),
    (12000, 50, 30000),
])
def test_item_split_shapes(qieo, oracle_mod, ng, n_pop, wmax):
    inst = workloads.random_instance(ng, n_pop, seed=400 + ng % 97, wmax=wmax)
    assert (int(inst.values.max()) <= (1 << 14) - 1) == (wmax <= 16378)
    g, o = _pair(qieo, oracle_mod, inst)
    for n in (1, 5, 12):
        path = _step_path(g, n)
        o.run(n)
        assert path == (qieo.PATH_ONCHIP, 1), "%d x %d: call of %d ran as %s" % (n_pop, ng, n, path)
        assert_state_equal(g, o, label="%d x %d after %d" % (n_pop, ng, o.t))
    say("  %d x %d: 18 generations in three calls equal the oracle" % (n_pop, ng))
    g.close()


def test_mixed_with_per_generation_launches_and_exports(qieo, oracle_mod):
    """On-chip calls interleaved with per-generation calls (mode 0), the
    default mode, exports in between, and a checkpoint resumed into a fresh
    handle that continues with per-generation launches."""
    inst = workloads.random_instance(5000, 700, seed=431)
    g, o = _pair(qieo, oracle_mod, inst)
    plan = [(3, 6), (0, 5), (3, 1), (1, 9), (0, 2), (3, 11)]
    for mode, n in plan:
        g.set_persistent(mode)
        g.step(n)
        assert g.call_path() == (qieo.PATH_LAUNCHES if mode == 0 else qieo.PATH_ONCHIP)
        o.run(n)
        assert_state_equal(g, o, label="mode %d, after %d" % (mode, o.t))
    snap = g.export_state()
    h = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    h.import_state(snap)
    h.set_persistent(0)
    g.set_persistent(3)
    for n in (4, 7):
        g.step(n)
        h.step(n)
        o.run(n)
    assert_state_equal(g, o, label="on-chip after resume point")
    assert_state_equal(h, o, label="resumed handle")
    say("  %d generations across modes, exports and a checkpoint" % o.t)
    g.close()
    h.close()


def test_default_mode_takes_it_for_calls_of_four_or_more(qieo, oracle_mod):
    inst = workloads.random_instance(10000, 1024, seed=432)
    g, o = _pair(qieo, oracle_mod, inst, mode=1)
    assert _step_path(g, 3) == (qieo.PATH_LAUNCHES, 3)     # below the threshold
    assert _step_path(g, 4) == (qieo.PATH_ONCHIP, 1)
    o.run(7)
    assert_state_equal(g, o, label="default mode")
    g.close()


@pytest.mark.parametrize("ng,n_pop,onchip", [
    (200, 256, True),      # 256 rows of one chunk
    (4000, 64, True),      # 1024 (row, chunk) items
    (5000, 24, True),      # rows of 20 chunks
    (1000, 128, False),    # 512 items, 128 rows: per-generation launches
    (1300, 96, False),     # 576 items
])
def test_default_mode_rule(qieo, oracle_mod, ng, n_pop, onchip):
    """Mode 1 takes the loop from 256 rows, 1024 items or rows of 20 chunks
    (calls of >= 4 generations); both sides of the rule equal the oracle."""
    inst = workloads.random_instance(ng, n_pop, seed=450 + ng % 31)
    g, o = _pair(qieo, oracle_mod, inst, mode=1)
    path, _ = _step_path(g, 6)
    assert path == (qieo.PATH_ONCHIP if onchip else qieo.PATH_LAUNCHES), (n_pop, ng, path)
    o.run(6)
    assert_state_equal(g, o, label="default mode %d x %d" % (n_pop, ng))
    g.close()


def test_populations_it_does_not_take_run_per_generation(qieo, oracle_mod):
    """Mode 3 on a population beyond its register budget (4096 x 5000:
    16 rows of 20 chunks per compute unit): per-generation launches, same
    results as the oracle."""
    inst = workloads.random_instance(5000, 4096, seed=433)
    g, o = _pair(qieo, oracle_mod, inst)
    assert _step_path(g, 5) == (qieo.PATH_LAUNCHES, 5)
    o.run(5)
    assert_state_equal(g, o, label="4096 x 5000, mode 3")
    g.close()


@pytest.mark.parametrize("wmax,path", [(20, "onchip"), (30000, "launches")])
def test_long_rows_on_chip_only_with_packed_tables(qieo, oracle_mod, wmax, path):
    """40 x 30,000 (118 chunks a row, one row a workgroup): its item tables
    fit a workgroup's LDS only packed (items of at most 14 bits), so mode 3
    takes the on-chip loop for small items and per-generation launches for
    large ones; both equal the oracle."""
    inst = workloads.random_instance(30000, 40, seed=449, wmax=wmax)
    g, o = _pair(qieo, oracle_mod, inst)
    want = qieo.PATH_ONCHIP if path == "onchip" else qieo.PATH_LAUNCHES
    for n in (4, 9):
        got = _step_path(g, n)
        o.run(n)
        assert got == (want, 1 if path == "onchip" else n), (wmax, n, got)
        assert_state_equal(g, o, label="40 x 30000, items up to %d, after %d" % (wmax, o.t))
    g.close()


# (n_items, n_pop, seed, window, calls, mode): where the oracle stops is
# noted per case; the calls put the stop mid-call, at a call's last
# generation (found by the finish, the next call then runs nothing), and
# after a run of equal elites that began in an earlier call (the run is
# seeded from the fitness ring).
@pytest.mark.parametrize("ng,n_pop,seed,window,calls,mode", [
    (3000, 1000, 441, 2, [10, 30, 40], 3),     # stops after 67, in the third call
    (3000, 1000, 441, 2, [10, 30, 40], 1),     # the same calls in the default mode
    (700, 2000, 442, 3, [1, 50, 200], 3),      # 136
    (9000, 300, 443, 2, [13, 5], 3),           # 13: the first call's finish
    (500, 600, 447, 3, [40, 30], 3),           # 42: the run began in the first call
    (256, 1024, 448, 3, [100, 100], 3),        # 136
    (256, 1024, 448, 1, [5, 5], 3),            # window 1: every elite completes it
    (60, 4000, 446, 8, [4, 4, 100], 3),        # 65
    (12000, 50, 445, 2, [7, 50], 3),           # 23
])
def test_convergence_window_stops_with_the_oracle(qieo, oracle_mod, ng, n_pop, seed, window,
                                                  calls, mode):
    inst = workloads.random_instance(ng, n_pop, seed=seed)
    g, o = _pair(qieo, oracle_mod, inst, mode=mode)
    g.set_convergence(window)
    n = o.run_until_converged(sum(calls), window)
    assert o.converged(window), "the case is meant to converge"
    for c in calls:
        assert _step_path(g, c) == (qieo.PATH_ONCHIP, 1), "call of %d" % c
    conv, at = g.converged()
    assert (g.generations, conv, at) == (n, 1, n - 1)
    assert_state_equal(g, o, label="%d x %d, window %d" % (n_pop, ng, window))
    g.step(6)                                  # nothing runs after convergence
    assert g.call_path() == qieo.PATH_ONCHIP and g.generations == n
    assert_state_equal(g, o, label="%d x %d, window %d, after" % (n_pop, ng, window))
    say("  %d x %d, window %d: stops after %d generations with the oracle" % (n_pop, ng, window, n))
    g.close()


def test_barrier_timeout_ends_the_launch_and_is_reported(qieo):
    """A zero bound on the grid-barrier wait: the workgroups give up at the
    first barrier that is not already complete, every one of them leaves
    the launch, and qieo_sync reports QIEO_EDEVICE.  A fresh instance on the
    same device runs normally afterwards."""
    inst = workloads.random_instance(3000, 1000, seed=435)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_persistent(3)
    g.set_barrier_timeout(0)
    with pytest.raises(qieo.QieoError) as ei:
        g.step(50)
    assert ei.value.code == qieo.QIEO_EDEVICE and "barrier" in str(ei.value)
    g.close()
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_persistent(3)
    g.step(5)
    assert g.call_path() == qieo.PATH_ONCHIP and g.generations == 5
    g.close()
    with pytest.raises(qieo.QieoError):
        qieo.Instance(inst.values, inst.weights, inst.capacity, 1, 1).set_barrier_timeout(-1)


def test_convergence_across_a_checkpoint(qieo, oracle_mod):
    """A run of equal elites that spans a checkpoint: the state exported
    after generation 40 (window 3, the oracle stops after 42) is imported
    into a fresh handle, whose on-chip call seeds its run from the restored
    fitness ring and stops where the oracle does; the original handle,
    continued with per-generation launches, stops there too."""
    inst = workloads.random_instance(500, 600, seed=447)
    g, o = _pair(qieo, oracle_mod, inst)
    g.set_convergence(3)
    n = o.run_until_converged(100, 3)
    assert (n, o.converged(3)) == (42, True)
    assert _step_path(g, 40) == (qieo.PATH_ONCHIP, 1)
    snap = g.export_state()
    h = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    h.import_state(snap)
    h.set_persistent(3)
    assert _step_path(h, 30) == (qieo.PATH_ONCHIP, 1)
    g.set_persistent(0)
    assert _step_path(g, 30)[0] == qieo.PATH_LAUNCHES
    for x, label in ((h, "imported, on-chip"), (g, "original, launches")):
        assert (x.generations,) + tuple(x.converged()) == (n, 1, n - 1), label
        assert_state_equal(x, o, label=label)
    g.close()
    h.close()


def test_concurrent_instances_on_their_own_streams(qieo, oracle_mod):
    """Three instances, each on its own stream, whose calls take the on-chip
    loop and are enqueued back to back before any is waited for: every
    cooperative launch completes (a grid that could not be co-resident
    would end at the barrier bound with QIEO_EDEVICE, not hang), and each
    instance equals its oracle."""
    insts = [workloads.random_instance(3000, 512, seed=460 + k) for k in range(3)]
    gs, os_ = [], []
    for inst in insts:
        g, o = _pair(qieo, oracle_mod, inst, mode=3)
        g.set_barrier_timeout(5_000_000)
        gs.append(g)
        os_.append(o)
    for _ in range(3):
        for g in gs:
            g.step_async(7)
    for g, o in zip(gs, os_):
        g.sync()
        assert g.call_path() == qieo.PATH_ONCHIP
        o.run(21)
        assert_state_equal(g, o, label="concurrent instance")
        g.close()
