"""Checkpoint and resume: a population exported after some generations and
loaded into a fresh handle of the same problem continues bit for bit, as
the uninterrupted run and the oracle do; snapshots of another problem are
refused without touching the handle."""
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


def _new(qieo, inst, precision=32):
    return qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                         precision=precision)


def _same(a, b, label):
    x, y = a.export_rows(), b.export_rows()
    for key in ("alpha", "beta", "alleles", "fitness", "profit", "weight"):
        assert np.array_equal(x[key], y[key]), (label, key)
    assert x["elite"] == y["elite"], label
    ra, rb = a.best(), b.best()
    assert (ra.fitness, ra.profit, ra.weight, ra.generation, ra.chromosome) == \
        (rb.fitness, rb.profit, rb.weight, rb.generation, rb.chromosome), label
    assert np.array_equal(ra.alleles(a.n_items), rb.alleles(b.n_items)), label


@pytest.mark.parametrize("ng,n_pop,before,after", [(100, 16, 7, 9), (1000, 33, 1, 12),
                                                   (4097, 20, 25, 5), (300, 9, 0, 6)])
def test_resume_continues_the_trajectory(qieo, oracle_mod, ng, n_pop, before, after):
    inst = workloads.random_instance(ng, n_pop, seed=300 + ng)
    say("resume Ng=%d Np=%d after %d generations" % (ng, n_pop, before))
    a = _new(qieo, inst)
    a.step(before)
    snap = a.export_state()
    b = _new(qieo, inst)
    b.step(3)                                   # its own state is replaced
    b.import_state(snap)
    assert b.generations == before
    if before:
        _same(a, b, "right after import")
    a.step(after)
    b.step(after)
    _same(a, b, "resumed")
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(before + after)
    assert_state_equal(b, o, label="resumed vs oracle")


def test_resume_keeps_the_convergence_history(qieo, oracle_mod):
    inst = workloads.small_instance()
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    window = 20
    ran = o.run_until_converged(5000, window)
    assert o.converged(window) and ran > window     # 1218 generations for this instance
    cut = ran - 7                               # the window spans the checkpoint
    a = _new(qieo, inst)
    a.set_convergence(window)
    a.step(cut)
    assert not a.converged()[0]
    b = _new(qieo, inst)
    b.import_state(a.export_state())
    b.step(5000)
    conv, gen = b.converged()
    assert conv and gen == ran - 1, (conv, gen, ran)
    assert b.generations == ran
    assert_state_equal(b, o, label="converged after resume")


def test_resume_binary64(qieo, oracle_mod):
    inst = workloads.random_instance(700, 12, seed=77)
    a = _new(qieo, inst, 64)
    a.step(6)
    b = _new(qieo, inst, 64)
    b.import_state(a.export_state())
    b.step(8)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=64)
    o.run(14)
    assert_state_equal(b, o, label="binary64 resumed")


def test_foreign_snapshots_are_refused(qieo):
    inst = workloads.random_instance(500, 8, seed=5)
    a = _new(qieo, inst)
    a.step(4)
    snap = a.export_state()
    b = _new(qieo, inst)
    b.step(2)
    before = b.export_rows()
    others = [
        workloads.random_instance(500, 8, seed=6),                  # other items and seed
        workloads.random_instance(500, 9, seed=5),                  # other population size
    ]
    for other in others:
        c = _new(qieo, other)
        with pytest.raises(qieo.QieoError) as ei:
            c.import_state(snap)
        assert ei.value.code == qieo.QIEO_EINVAL
    d = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed + 1)
    with pytest.raises(qieo.QieoError):
        d.import_state(snap)                                        # other seed only
    e = _new(qieo, inst, 64)
    with pytest.raises(qieo.QieoError):
        e.import_state(snap)                                        # other precision
    for bad in (snap[:100], snap[:-1]):
        with pytest.raises(qieo.QieoError):
            b.import_state(bad)                                     # truncated
    corrupt = snap.copy()
    corrupt[0] ^= 1
    with pytest.raises(qieo.QieoError):
        b.import_state(corrupt)                                     # not a snapshot
    # an elite key naming a row outside the population: the 64-bit key is
    # (fitness ^ 2^31) << 32 | ~row; find it in the arena image (8-byte
    # aligned after the 64-byte header) and point it at row n_pop
    rows = a.export_rows()
    e_row, f_e = rows["elite"], int(rows["fitness"][rows["elite"]])
    key = (((f_e & 0xFFFFFFFF) ^ 0x80000000) << 32) | (~e_row & 0xFFFFFFFF)
    words = snap[64:64 + (snap.size - 64) // 8 * 8].view("<u8")
    hits = np.flatnonzero(words == np.uint64(key))
    assert hits.size >= 1
    bad_key = snap.copy()
    bad_words = bad_key[64:64 + words.size * 8].view("<u8")
    bad_words[hits] = (bad_words[hits] & np.uint64(0xFFFFFFFF00000000)) | \
        np.uint64(~inst.n_pop & 0xFFFFFFFF)
    with pytest.raises(qieo.QieoError) as ei:
        b.import_state(bad_key)                                     # elite row out of range
    assert ei.value.code == qieo.QIEO_EINVAL
    after = b.export_rows()
    for key in ("alpha", "beta", "alleles", "fitness"):
        assert np.array_equal(before[key], after[key]), key
    assert b.generations == 2
