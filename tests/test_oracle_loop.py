"""Whole-loop pins of the oracle: invariants that any correct QIEO run on
these readings satisfies, checked against exact knapsack references."""
import math

import numpy as np
import pytest

import workloads


def _run_checking_norm(o, n, tol=1e-5):
    worst = 0.0
    for _ in range(n):
        o.generation()
        a, b = o.amplitudes()
        dev = np.abs(a.astype(np.float64) ** 2 + b.astype(np.float64) ** 2 - 1.0).max()
        worst = max(worst, float(dev))
        assert dev <= tol
    return worst


def test_norm_invariant_every_generation_small_instance(oracle_mod):
    inst = workloads.small_instance()
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    worst = _run_checking_norm(o, inst.generations)
    assert worst < 1e-6


def test_norm_invariant_long_run_many_rotations(oracle_mod):
    inst = workloads.random_instance(300, 64, seed=31)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    _run_checking_norm(o, 1500)


def test_best_is_monotone_feasible_and_bounded_by_dp(oracle_mod):
    inst = workloads.small_instance()
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    opt = oracle_mod.knap_dp(inst.values, inst.weights, inst.capacity)
    lp = oracle_mod.knap_lp_bound(inst.values, inst.weights, inst.capacity)
    assert opt <= lp + 1e-9
    prev = None
    for g in range(inst.generations):
        o.generation()
        b = o.best()
        assert b.has_best
        if prev is not None:
            assert b.fitness >= prev
        prev = b.fitness
        assert b.fitness <= opt
        bits = b.bits.astype(np.int64)
        assert int(bits @ inst.values) == b.profit
        assert int(bits @ inst.weights) == b.weight
        if b.weight <= inst.capacity:
            assert b.fitness == b.profit
        else:
            assert b.fitness == -(b.weight - inst.capacity)
    # the run improves a lot on the all-random start and is feasible
    assert o.best().weight <= inst.capacity
    assert o.best().fitness > 0.8 * opt


def test_bruteforce_optimum_equals_dp(oracle_mod):
    for seed in range(6):
        inst = workloads.random_instance(18, 4, seed=100 + seed)
        bf, m = oracle_mod.knap_bruteforce(inst.values, inst.weights, inst.capacity)
        assert bf == oracle_mod.knap_dp(inst.values, inst.weights, inst.capacity)
        bits = (m >> np.arange(18)) & 1
        assert int(bits @ inst.weights) <= inst.capacity


def test_best_found_reaches_enumeration_optimum_on_tiny_instance(oracle_mod):
    inst = workloads.random_instance(16, 32, seed=7)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(300)
    bf, _ = oracle_mod.knap_bruteforce(inst.values, inst.weights, inst.capacity)
    assert o.best().fitness <= bf
    assert o.best().fitness >= bf - 10


def _snapshot(o):
    a, b = o.amplitudes()
    f, P, W = o.fitness()
    bb = o.best()
    return dict(a=a, b=b, x=o.alleles(), P=P, W=W, e=o.elite, t=o.t,
                best=(bb.fitness, bb.profit, bb.weight, bb.generation, bb.chromosome),
                bits=bb.bits, f=f)


def test_penalty_factor_does_not_change_the_trajectory(oracle_mod):
    """Any lambda > 0 orders every pair of fitnesses the same way (feasible
    >= 0 > infeasible, infeasible ordered by excess), so only the reported
    infeasible values scale."""
    inst = workloads.random_instance(120, 24, seed=5)
    o1 = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed, lam=1)
    o7 = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed, lam=7)
    saw_infeasible = False
    for _ in range(60):
        o1.generation()
        o7.generation()
        s1, s7 = _snapshot(o1), _snapshot(o7)
        for k in ("a", "b", "x", "P", "W", "bits"):
            assert np.array_equal(s1[k], s7[k]), k
        assert s1["e"] == s7["e"]
        inf = s1["W"] > inst.capacity
        saw_infeasible |= bool(inf.any())
        assert np.array_equal(s7["f"][inf], 7 * s1["f"][inf])
        assert np.array_equal(s7["f"][~inf], s1["f"][~inf])
    assert saw_infeasible


def test_split_runs_equal_one_run(oracle_mod):
    inst = workloads.random_instance(77, 10, seed=9)
    a = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    b = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    a.run(40)
    b.run(13)
    b.run(27)
    sa, sb = _snapshot(a), _snapshot(b)
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k


def test_seed_determines_the_trajectory(oracle_mod):
    inst = workloads.random_instance(64, 8, seed=3)
    a = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, 5)
    b = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, 5)
    c = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, 6)
    for o in (a, b, c):
        o.run(20)
    assert np.array_equal(a.amplitudes()[1], b.amplitudes()[1])
    assert not np.array_equal(a.amplitudes()[1], c.amplitudes()[1])


def test_row_threads_give_identical_state(oracle_mod):
    inst = workloads.random_instance(333, 37, seed=12)
    a = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    b = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          threads=4)
    a.run(30)
    b.run(30)
    sa, sb = _snapshot(a), _snapshot(b)
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k


def test_population_converges_toward_the_elite(oracle_mod):
    """After many generations most amplitudes sit near a pole and the
    population agrees with its elite on most genes."""
    inst = workloads.random_instance(200, 32, seed=21)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(1000)
    _, b = o.amplitudes()
    b2 = b.astype(np.float64) ** 2
    assert np.mean((b2 < 0.05) | (b2 > 0.95)) > 0.6
    x = o.alleles()
    assert np.mean(x == x[o.elite][None, :]) > 0.85


def test_quality_report_small_instance(oracle_mod, capsys):
    inst = workloads.small_instance()
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o.run(inst.generations)
    opt = oracle_mod.knap_dp(inst.values, inst.weights, inst.capacity)
    gap = (opt - o.best().fitness) / opt
    print("small instance: best %d, DP optimum %d, gap %.4f" % (o.best().fitness, opt, gap))
    assert 0 <= gap < 0.2


def test_convergence_window_stops_at_first_stable_window(oracle_mod):
    """Sec. IV-A: stop once the elite fitness has been one value for `window`
    generations.  The stopping point is recomputed here from the per-
    generation elite fitness of an identical run."""
    inst = workloads.small_instance()
    for window in (2, 5, 20):
        o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
        n = o.run_until_converged(5000, window)
        ref = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
        hist = []
        stop = None
        for g in range(5000):
            ref.generation()
            hist.append(int(ref.fitness()[0].max()))
            if len(hist) >= window and len(set(hist[-window:])) == 1:
                stop = g + 1
                break
        assert stop is not None and n == stop, (window, n, stop)
        assert o.converged(window)
        assert o.run_until_converged(100, window) == 0      # nothing more once converged
        assert o.t == stop


def test_convergence_window_respects_the_cap(oracle_mod):
    inst = workloads.random_instance(300, 64, seed=31)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    assert o.run_until_converged(40, 20) == 40
    assert not o.converged(20)
    assert not o.converged(0)


@pytest.mark.parametrize("precision", [32, 64])
def test_row_generation_composes_to_the_population_oracle(oracle_mod, precision):
    """Every chromosome driven through the chromosome-local step, with
    DetermineElite taken over the rows' fitness (largest, lowest index),
    gives the population oracle's alleles, fitness, elite and amplitudes at
    every generation (ragged Ng, rows below, at and above the elite)."""
    inst = workloads.random_instance(301, 9, seed=4)
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=precision)
    bits = np.uint64 if precision == 64 else np.uint32
    a0, b0 = o.amplitudes()
    rows = [{"a": a0[c].copy(), "b": b0[c].copy(), "x": None, "f": None}
            for c in range(inst.n_pop)]
    elite_x, fe = None, None
    for t in range(30):
        prev_a, prev_b = o.amplitudes()          # as generation t will observe them
        o.run(1)
        x_o = o.alleles()
        f_o, P_o, W_o = o.fitness()
        for c, r in enumerate(rows):
            below = t > 0 and r["f"] < fe
            a, b, x, f, P, W = oracle_mod.row_generation(
                inst.seed, t, c, inst.values, inst.weights, inst.capacity, r["a"], r["b"],
                r["x"], elite_x, below, precision=precision)
            assert np.array_equal(a.view(bits), prev_a[c].view(bits)), (t, c)
            assert np.array_equal(b.view(bits), prev_b[c].view(bits)), (t, c)
            assert np.array_equal(x, x_o[c]), (t, c)
            assert (f, P, W) == (f_o[c], P_o[c], W_o[c]), (t, c)
            r.update(a=a, b=b, x=x, f=f)
        fits = [r["f"] for r in rows]
        e = int(np.argmax(fits))
        assert e == o.elite
        elite_x, fe = rows[e]["x"], rows[e]["f"]
