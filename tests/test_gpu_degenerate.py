"""Degenerate instances and the real serving stream against the oracle.

Degenerate cases: nothing fits (capacity 0), everything fits (capacity at
or above the total weight), all values zero (every feasible string ties, so
the elite is decided by the lowest-index rule alone), identical items, a
single gene, a single chromosome, and item values whose sums reach the int32
limit.  The serving stream: the first requests of the Poisson workload run
through the continuous-batching server; the smallest are compared with the
oracle bit for bit, all of them with what holds at any size."""
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


def _inst(values, weights, capacity, n_pop, seed):
    v = np.asarray(values, np.int32)
    w = np.asarray(weights, np.int32)
    return workloads.Instance(v, w, int(capacity), int(n_pop), int(seed), 10, name="degenerate")


def _cases():
    r = np.random.default_rng(7)
    w300 = r.integers(1, 50, 300)
    return {
        "capacity 0": _inst(r.integers(1, 20, 300), w300, 0, 19, 1),
        "capacity >= total weight": _inst(r.integers(1, 20, 300), w300, int(w300.sum()), 19, 2),
        "all values zero": _inst(np.zeros(300), w300, int(w300.sum()) // 2, 23, 3),
        "identical items": _inst(np.full(500, 7), np.full(500, 3), 600, 17, 4),
        "single gene": _inst([5], [3], 3, 9, 5),
        "single gene, never fits": _inst([5], [3], 2, 9, 6),
        "single chromosome": _inst(r.integers(1, 20, 777), r.integers(1, 20, 777), 3000, 1, 7),
        "int32 sums": _inst([1_000_000_000, 1_000_000_000, 147_483_647, 0],
                            [1_000_000_000, 1_000_000_000, 147_483_647, 0], 2_000_000_000, 12, 8),
    }


@pytest.mark.parametrize("name", list(_cases().keys()))
@pytest.mark.parametrize("persistent", [0, 1])
def test_degenerate_instances_follow_the_oracle(qieo, oracle_mod, name, persistent):
    inst = _cases()[name]
    say("degenerate: %s (persistent mode %d)" % (name, persistent))
    g = qieo.Instance(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    g.set_persistent(persistent)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    for n in (1, 1, 5, 40):
        g.step(n)
        o.run(n)
        assert_state_equal(g, o, label="%s t=%d" % (name, o.t))
    f, _, W = o.fitness()
    b = g.best()
    if name == "capacity 0":                 # only the empty string is feasible
        assert (f == -W).all() and b.fitness == -b.weight
    if name == "capacity >= total weight":
        assert (f >= 0).all() and b.feasible
    if name == "all values zero":
        assert b.fitness == 0
