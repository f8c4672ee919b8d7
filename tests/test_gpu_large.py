"""Parity at sizes beyond the workloads: a population past 2^32 genes, rows
of the maximum length the library accepts, and an export of more rows than
one grid dimension holds.  (The whole-population checks of the largest
workload are in test_gpu_full_population.py.)"""
import os

import numpy as np
import pytest

import workloads
from gpu_common import assert_state_equal, bits_equal, say

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def qieo():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2609_30862_amd import qieo as q
    return q


def test_population_beyond_2_32_genes(qieo, oracle_mod):
    """32,768 chromosomes x 131,136 genes = 4.297e9 genes, past 2^32 (34 GB of
    binary32 amplitudes), in the streaming launch configuration.  Only
    DetermineElite looks across chromosomes, so each sampled chromosome, each
    generation's elite and the elites' own histories are recomputed one
    chromosome at a time by the oracle, given the GPU's elite sequence; that
    sequence is checked against the argmax (lowest index) of the GPU's
    fitness array, whose sampled entries must equal the oracle's."""
    n_pop, ng = 32768, 131136
    pitch = (ng + 63) // 64 * 64
    assert n_pop * pitch > 2 ** 32
    inst = workloads.random_instance(ng, n_pop, seed=9)
    say("population of %d x %d = %.4g genes" % (n_pop, ng, n_pop * ng))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    say("  variant bits %d" % g.kernel_flags())
    tiny = oracle_mod.Oracle(inst.values[:1], inst.weights[:1], 1, 1, inst.seed)
    a0 = np.full(ng, tiny.amplitudes()[0][0, 0], dtype=np.float32)   # the initial amplitude
    del tiny
    seed, v, w, cap = inst.seed, inst.values, inst.weights, inst.capacity
    hist = {}       # chromosome -> per generation (alpha, beta as observed, alleles, fitness)
    elites = []     # per generation: (row, fitness) from the GPU

    def state(c, k):
        h = hist.setdefault(c, [])
        while len(h) <= k:
            t = len(h)
            if t == 0:
                a, b, x, f, _, _ = oracle_mod.row_generation(seed, 0, c, v, w, cap, a0, a0)
            else:
                e, fe = elites[t - 1]
                ex = state(e, t - 1)[2]
                pa, pb, px, pf = h[t - 1]
                a, b, x, f, _, _ = oracle_mod.row_generation(seed, t, c, v, w, cap, pa, pb,
                                                             px, ex, pf < fe)
            h.append((a, b, x, f))
        return h[k]

    sample = [0, 1, 2, 4095, 16384, 30001, 32766, 32767]
    for k in range(3):
        g.step(1)
        st = g.export_rows(0, n_pop, amplitudes=False, alleles=False)
        fit = st["fitness"].astype(np.int64)
        e = int(st["elite"])
        assert e == int(np.argmax(fit))
        elites.append((e, int(fit[e])))
        for c in sorted(set(sample + [e])):
            a, b, x, f = state(c, k)
            assert f == fit[c], "generation %d row %d" % (k, c)
            ex = state(e, k)[2]
            # amplitudes after CIP(k), as the export applies the pending rotation
            ra, rb, _, _, _, _ = oracle_mod.row_generation(seed, k + 1, c, v, w, cap, a, b, x,
                                                           ex, f < fit[e])
            s = g.export_rows(c, 1)
            assert np.array_equal(s["alleles"][0], x), "alleles, generation %d row %d" % (k, c)
            assert bits_equal(s["alpha"][0], ra) and bits_equal(s["beta"][0], rb), \
                "amplitudes, generation %d row %d" % (k, c)
        say("  generation %d: elite %d, fitness %d, %d rows checked" % (k, e, fit[e],
                                                                      len(set(sample + [e]))))
    g.close()


def test_rows_of_the_maximum_length(qieo, oracle_mod):
    """Two chromosomes of 2^30 - 256 genes, the longest row the library
    accepts (17 GB of binary32 amplitudes, segment order): both rows'
    alleles, fitness and rotated amplitudes over two generations equal the
    oracle's chromosome-by-chromosome step, and the elite is the argmax.
    Values and weights in {1, 2} keep both sums within int32."""
    from concurrent.futures import ThreadPoolExecutor
    ng, n_pop, seed = (1 << 30) - 256, 2, 11
    v, w, cap = workloads.independent_items(ng, 1, 2, seed=seed)
    assert int(v.sum(dtype=np.int64)) < 2 ** 31 and int(w.sum(dtype=np.int64)) < 2 ** 31
    say("rows of %d genes x %d" % (ng, n_pop))
    g = qieo.Instance(v, w, cap, n_pop, seed)
    assert g.kernel_flags() & 16                       # streaming: segment order
    tiny = oracle_mod.Oracle(v[:1], w[:1], 1, 1, seed)
    a0 = tiny.amplitudes()[0][0, 0]
    del tiny
    alpha = [np.full(ng, a0, dtype=np.float32) for _ in range(n_pop)]
    beta = [np.full(ng, a0, dtype=np.float32) for _ in range(n_pop)]
    none = np.zeros(ng, np.uint8)
    x = [[np.zeros(ng, np.uint8) for _ in range(n_pop)] for _ in range(2)]
    fit = [[0] * n_pop for _ in range(2)]

    def oracle_step(t, c, x_prev, elite_x, below):
        return oracle_mod.row_generation_inplace(seed, t, c, v, w, cap, alpha[c], beta[c],
                                                 x_prev, elite_x, below, x[t][c])[0]

    with ThreadPoolExecutor(n_pop) as pool:
        # generation 0: observation and Evaluation only
        g.step(1)
        st = g.export_rows(0, n_pop, amplitudes=False, alleles=False)
        fit[0] = list(pool.map(lambda c: oracle_step(0, c, none, none, False), range(n_pop)))
        assert list(st["fitness"]) == fit[0]
        e0 = int(np.argmax(fit[0]))
        assert st["elite"] == e0
        held = []
        for c in range(n_pop):
            s = g.export_rows(c, 1)                   # amplitudes after CIP(0)
            assert np.array_equal(s["alleles"][0], x[0][c]), "alleles, generation 0 row %d" % c
            held.append((s["alpha"][0], s["beta"][0]))
            del s
        say("  generation 0: fitness %s, elite %d" % (fit[0], e0))
        # generation 1: CIP(0) toward the elite's alleles, then QIP and Evaluation
        fit[1] = list(pool.map(lambda c: oracle_step(1, c, x[0][c], x[0][e0],
                                                     fit[0][c] < fit[0][e0]), range(n_pop)))
        for c in range(n_pop):
            assert bits_equal(held[c][0], alpha[c]) and bits_equal(held[c][1], beta[c]), \
                "amplitudes after CIP(0), row %d" % c
        del held
        g.step(1)
        st = g.export_rows(0, n_pop, amplitudes=False, alleles=False)
        assert list(st["fitness"]) == fit[1]
        assert st["elite"] == int(np.argmax(fit[1]))
        for c in range(n_pop):
            s = g.export_rows(c, 1, amplitudes=False)
            assert np.array_equal(s["alleles"][0], x[1][c]), "alleles, generation 1 row %d" % c
            del s
        say("  generation 1: fitness %s" % fit[1])
    g.close()


def test_export_of_more_rows_than_one_grid_dimension_holds(qieo, oracle_mod):
    """70,001 chromosomes of 50 genes: one export call of every row with
    amplitudes and alleles (more rows than a grid's y dimension takes, so
    the library exports them in blocks) equals the oracle's state, after
    1 and 4 generations."""
    inst = workloads.random_instance(50, 70_001, seed=13)
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=min(16, os.cpu_count() or 1))
    for gens in (1, 3):
        g.step(gens)
        o.run(gens)
        assert_state_equal(g, o, label="70,001 rows after %d generations" % o.t)
    g.close()
