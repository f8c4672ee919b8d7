"""Helpers shared by the GPU tests: bit-exact comparison of a libqieo
instance's exported state with the CPU oracle's state."""
import sys

import numpy as np


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def _bits(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    return a.dtype == b.dtype and np.array_equal(_bits(a), _bits(b))


def assert_state_equal(inst, orc, rows=None, label=""):
    """Every row in `rows` (default all): amplitudes bit for bit, alleles,
    profit, weight and fitness; plus elite index and best-so-far record."""
    np_ = inst.n_pop
    rows = np.arange(np_) if rows is None else np.asarray(rows)
    a_o, b_o = orc.amplitudes()
    x_o = orc.alleles()
    f_o, P_o, W_o = orc.fitness()
    # contiguous runs keep the number of export calls small
    runs = []
    start = prev = int(rows[0])
    for r in rows[1:]:
        r = int(r)
        if r == prev + 1:
            prev = r
            continue
        runs.append((start, prev + 1))
        start = prev = r
    runs.append((start, prev + 1))
    elite = None
    for (r0, r1) in runs:
        st = inst.export_rows(r0, r1 - r0)
        elite = st["elite"]
        sl = slice(r0, r1)
        if not bits_equal(st["alpha"], a_o[sl]) or not bits_equal(st["beta"], b_o[sl]):
            bad = np.argwhere((_bits(st["alpha"]) != _bits(a_o[sl])) |
                              (_bits(st["beta"]) != _bits(b_o[sl])))
            r, i = bad[0]
            raise AssertionError(
                "%s amplitudes differ at row %d gene %d: gpu (%r, %r) oracle (%r, %r); %d genes"
                % (label, r0 + r, i, st["alpha"][r, i], st["beta"][r, i], a_o[r0 + r, i],
                   b_o[r0 + r, i], len(bad)))
        if not np.array_equal(st["alleles"], x_o[sl]):
            bad = np.argwhere(st["alleles"] != x_o[sl])
            raise AssertionError("%s alleles differ at %s (%d genes)" % (label, bad[0], len(bad)))
        assert np.array_equal(st["profit"].astype(np.int64), P_o[sl]), label + " profit"
        assert np.array_equal(st["weight"].astype(np.int64), W_o[sl]), label + " weight"
        assert np.array_equal(st["fitness"].astype(np.int64), f_o[sl]), label + " fitness"
    assert elite == orc.elite, "%s elite gpu %d oracle %d" % (label, elite, orc.elite)
    gb = inst.best()
    ob = orc.best()
    assert (gb.fitness, gb.profit, gb.weight, gb.generation, gb.chromosome) == \
        (ob.fitness, ob.profit, ob.weight, ob.generation, ob.chromosome), \
        "%s best gpu %r oracle %r" % (label, gb, ob)
    assert np.array_equal(gb.alleles(inst.n_items), ob.bits), label + " best bits"
