"""Pins of the oracle's four generation steps against facts fixed outside it:
hand-worked values of eq. (1), brute-force enumeration, the knapsack dynamic
program, closed-form rotation angles and the geometry of the rotation gate."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
A0 = np.float32(1.0 / math.sqrt(2.0))


def f32(hexstr):
    return np.float32(float.fromhex(hexstr))


C_ROT = f32("0x1.ffbf52p-1")
S_ROT = f32("0x1.015122p-5")


# ----------------------------------------------------------------- constants
def test_rotation_constants_are_binary32_cos_sin_of_pi_over_100():
    assert C_ROT == np.float32(math.cos(0.01 * math.pi))
    assert S_ROT == np.float32(math.sin(0.01 * math.pi))
    assert f32("0x1.6a09e6p-1") == np.float32(1.0 / math.sqrt(2.0))


# ----------------------------------------------------------------- QIP
def _pop(oracle_mod, ng, n_pop, seed=11, cap=None):
    v = np.arange(1, ng + 1, dtype=np.int32)
    w = np.arange(1, ng + 1, dtype=np.int32)
    cap = int(w.sum() // 2) if cap is None else cap
    return oracle_mod.Oracle(v, w, cap, n_pop, seed)


def test_qip_initial_population_observes_about_half(oracle_mod):
    o = _pop(oracle_mod, 500, 40)
    o.qip()
    x = o.alleles()
    # beta^2 = fl(A0*A0) ~ 0.5: binomial mean within 6 sigma
    n = x.size
    assert abs(x.mean() - 0.5) < 6 * math.sqrt(0.25 / n)


def test_qip_reads_beta_not_alpha(oracle_mod):
    o = _pop(oracle_mod, 64, 8)
    ones = np.ones((8, 64), np.float32)
    zeros = np.zeros((8, 64), np.float32)
    o.set_amplitudes(zeros, ones)          # |1>: beta = 1
    o.qip()
    assert o.alleles().all()
    o.set_amplitudes(ones, zeros)          # |0>: beta = 0
    o.qip()
    assert not o.alleles().any()
    o.set_amplitudes(zeros, -ones)         # sign of beta does not matter
    o.qip()
    assert o.alleles().all()


@pytest.mark.parametrize("p", [0.05, 0.3, 0.5, 0.9])
def test_qip_frequency_matches_beta_squared(oracle_mod, p):
    ng, n_pop = 1000, 50
    o = _pop(oracle_mod, ng, n_pop, seed=int(p * 1000))
    b = np.full((n_pop, ng), np.float32(math.sqrt(p)), np.float32)
    a = np.full((n_pop, ng), np.float32(math.sqrt(1 - p)), np.float32)
    o.set_amplitudes(a, b)
    o.qip()
    q = float(np.float32(b[0, 0]) * np.float32(b[0, 0]))
    n = ng * n_pop
    assert abs(o.alleles().mean() - q) < 6 * math.sqrt(q * (1 - q) / n)


def test_qip_threshold_is_the_draw(oracle_mod):
    """x = 1 exactly when the draw's top 24 bits fall below beta^2 * 2^24."""
    ng, n_pop, seed = 256, 4, 77
    o = _pop(oracle_mod, ng, n_pop, seed=seed)
    b = np.full((n_pop, ng), np.float32(0.5), np.float32)  # beta^2 = 2^-2 exactly
    o.set_amplitudes(b, b)
    o.qip()
    x = o.alleles()
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for c in range(n_pop):
        for k in range(ng // 4):
            wds = oracle_mod.philox4x32_10([k, c, 0, 0], key)
            for j in range(4):
                assert x[c, 4 * k + j] == ((int(wds[j]) >> 8) < (1 << 22))


def test_qip_comparison_is_strict(oracle_mod):
    """At beta^2 == u exactly the allele is 0; one ulp more gives 1."""
    # find a seed whose first draw is q^2 * 2^-24 with q integer, so that
    # beta = q * 2^-12 squares exactly onto the draw
    found = None
    for seed in range(200000):
        m = int(round(oracle_mod.uniform(seed, 0, 0, 0) * 2**24))
        q = int(math.isqrt(m))
        if q * q == m and q > 0:
            found = (seed, q)
            break
    assert found is not None
    seed, q = found
    beta = np.float32(q * 2.0**-12)
    assert float(beta * beta) == oracle_mod.uniform(seed, 0, 0, 0)
    v = np.ones(4, np.int32)
    o = oracle_mod.Oracle(v, v, 2, 1, seed)
    a = np.full((1, 4), np.float32(0.6), np.float32)
    bb = np.full((1, 4), beta, np.float32)
    o.set_amplitudes(a, bb)
    o.qip()
    assert o.alleles()[0, 0] == 0
    bb[0, 0] = np.nextafter(beta, np.float32(2.0))
    o.set_amplitudes(a, bb)
    o.qip()
    assert o.alleles()[0, 0] == 1


# ----------------------------------------------------------------- FE, eq. (1)
def _golden_fe():
    rows, items, opt = [], None, None
    with open(os.path.join(HERE, "golden", "fe_worked_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "items":
                v = [int(s) for s in parts[1].split(",")]
                w = [int(s) for s in parts[2].split(",")]
                items = (v, w, int(parts[3]))
            elif parts[0] == "optimum":
                opt = int(parts[1])
            else:
                rows.append((parts[0], *[int(s) for s in parts[1:]]))
    return items, rows, opt


@pytest.mark.parametrize("lam", [1, 3])
def test_fe_worked_example(oracle_mod, lam):
    (v, w, cap), rows, _ = _golden_fe()
    o = oracle_mod.Oracle(v, w, cap, len(rows), 0, lam=lam)
    x = np.array([[int(ch) for ch in r[0]] for r in rows], np.uint8)
    o.set_alleles(x)
    o.fe()
    fit, P, W = o.fitness()
    for k, r in enumerate(rows):
        assert P[k] == r[1] and W[k] == r[2]
        assert fit[k] == (r[3] if lam == 1 else r[4])


def test_fe_worked_example_optimum_by_dp_and_enumeration(oracle_mod):
    (v, w, cap), _, opt = _golden_fe()
    assert oracle_mod.knap_dp(v, w, cap) == opt
    assert oracle_mod.knap_bruteforce(v, w, cap)[0] == opt


@pytest.mark.parametrize("n,seed", [(6, 1), (10, 2), (12, 3)])
def test_fe_all_strings_match_enumeration_and_dp(oracle_mod, n, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(1, 30, n).astype(np.int32)
    v = (w + rng.integers(0, 10, n)).astype(np.int32)
    cap = int(w.sum() // 2)
    strings = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    o = oracle_mod.Oracle(v, w, cap, 1 << n, 0)
    o.set_alleles(strings)
    o.fe()
    fit, P, W = o.fitness()
    assert np.array_equal(fit, oracle_mod.knap_all_fitness(v, w, cap))
    assert fit.max() == oracle_mod.knap_dp(v, w, cap)
    assert np.array_equal(P, strings.astype(np.int64) @ v.astype(np.int64))
    assert np.array_equal(W, strings.astype(np.int64) @ w.astype(np.int64))


def test_fe_extremes(oracle_mod):
    rng = np.random.default_rng(4)
    n = 300
    w = rng.integers(1, 11, n).astype(np.int32)
    v = (w + 5).astype(np.int32)
    cap = int(w.sum() // 2)
    o = oracle_mod.Oracle(v, w, cap, 3, 0)
    x = np.zeros((3, n), np.uint8)
    x[1] = 1
    o.set_alleles(x)
    o.fe()
    fit, P, W = o.fitness()
    assert fit[0] == 0 and P[0] == 0 and W[0] == 0
    assert fit[1] == -(int(w.sum()) - cap)


# ----------------------------------------------------------------- DetermineElite
def test_de_ties_go_to_lowest_index(oracle_mod):
    o = _pop(oracle_mod, 8, 6)
    o.set_fitness([3, 7, 5, 7, 7, 1])
    o.de()
    assert o.elite == 1
    o.set_fitness([-5, -2, -9, -2, -3, -4])
    o.de()
    assert o.elite == 1
    o.set_fitness([4, 4, 4, 4, 4, 4])
    o.de()
    assert o.elite == 0
    o.set_fitness([0, 0, 0, 0, 0, 9])
    o.de()
    assert o.elite == 5


def test_de_best_changes_only_on_strict_improvement(oracle_mod):
    o = _pop(oracle_mod, 8, 4)
    o.set_fitness([3, 7, 7, 1])
    o.de()
    b = o.best()
    assert b.has_best and b.fitness == 7 and b.chromosome == 1
    o.set_fitness([7, 1, 1, 1])      # equal, not larger: record stays
    o.de()
    assert o.elite == 0 and o.best().chromosome == 1
    o.set_fitness([1, 1, 8, 1])
    o.de()
    assert o.best().chromosome == 2 and o.best().fitness == 8


def test_de_first_generation_always_records_even_if_negative(oracle_mod):
    o = _pop(oracle_mod, 8, 3)
    o.set_fitness([-9, -4, -6])
    o.de()
    b = o.best()
    assert b.has_best and b.fitness == -4 and b.chromosome == 1


# ----------------------------------------------------------------- CIP gate
def _angle(a, b):
    return math.atan2(float(b), float(a))


def test_cip_closed_form_angle_tracking(oracle_mod):
    """k same-direction rotations from pi/4 land on pi/4 +- k*phi,
    phi = atan2(S, C) of the binary32 constants, within rounding."""
    phi = math.atan2(float(S_ROT), float(C_ROT))
    for tgt, sgn in ((1, +1), (0, -1)):
        a, b = A0, A0
        for k in range(1, 25):        # stays inside the first quadrant
            a, b, rot = oracle_mod.cip_gene(a, b, tgt)
            assert rot
            th = math.pi / 4 + sgn * k * phi
            assert abs(float(a) - math.cos(th)) <= 2e-7 * k
            assert abs(float(b) - math.sin(th)) <= 2e-7 * k


@pytest.mark.parametrize("deg", [20, 70, 110, 160, 200, 250, 290, 340])
def test_cip_moves_beta_squared_toward_target_in_every_quadrant(oracle_mod, deg):
    th = math.radians(deg)
    a, b = np.float32(math.cos(th)), np.float32(math.sin(th))
    a1, b1, r1 = oracle_mod.cip_gene(a, b, 1)
    a0, b0, r0 = oracle_mod.cip_gene(a, b, 0)
    assert r1 and r0
    assert float(b1) ** 2 > float(b) ** 2
    assert float(b0) ** 2 < float(b) ** 2
    # magnitude of the step is 0.01*pi
    for aa, bb in ((a1, b1), (a0, b0)):
        d = (_angle(aa, bb) - th) % (2 * math.pi)
        d = min(d, 2 * math.pi - d)
        assert abs(d - 0.01 * math.pi) < 1e-5


def test_cip_on_axes(oracle_mod):
    one, zero = np.float32(1), np.float32(0)
    # already at the target pole: skipped
    assert oracle_mod.cip_gene(zero, one, 1)[2] is False
    assert oracle_mod.cip_gene(one, zero, 0)[2] is False
    assert oracle_mod.cip_gene(zero, -one, 1)[2] is False
    # at the opposite pole: rotated toward the target
    a, b, r = oracle_mod.cip_gene(zero, one, 0)
    assert r and float(b) ** 2 < 1.0
    a, b, r = oracle_mod.cip_gene(one, zero, 1)
    assert r and float(b) ** 2 > 0.0


def test_cip_newton_step_restores_norm(oracle_mod):
    for (a, b) in [(0.70, 0.70), (0.72, 0.71), (0.1, 0.98), (-0.5, 0.86)]:
        a, b = np.float32(a), np.float32(b)
        n0 = abs(float(a) ** 2 + float(b) ** 2 - 1)
        a1, b1, _ = oracle_mod.cip_gene(a, b, 1)
        n1 = abs(float(a1) ** 2 + float(b1) ** 2 - 1)
        assert n1 < max(n0 / 10, 1e-6)


def test_cip_population_rules(oracle_mod):
    """Only chromosomes below the elite rotate, only where they differ from
    the elite, and always toward the elite's allele."""
    rng = np.random.default_rng(8)
    ng, n_pop = 97, 12
    w = rng.integers(1, 11, ng).astype(np.int32)
    v = (w + 5).astype(np.int32)
    o = oracle_mod.Oracle(v, w, int(w.sum() // 2), n_pop, 5)
    th = rng.uniform(0, 2 * math.pi, (n_pop, ng))
    o.set_amplitudes(np.cos(th).astype(np.float32), np.sin(th).astype(np.float32))
    o.qip()
    o.fe()
    fit = o.fitness()[0].copy()
    fit[7] = fit.max()               # force a tie with the elite
    o.set_fitness(fit)
    o.de()
    e = o.elite
    x = o.alleles()
    a0, b0 = o.amplitudes()
    o.cip()
    a1, b1 = o.amplitudes()
    for c in range(n_pop):
        for i in range(ng):
            moved = (a1[c, i] != a0[c, i]) or (b1[c, i] != b0[c, i])
            should = fit[c] < fit[e] and x[c, i] != x[e, i]
            assert moved == should
            if should:
                if x[e, i]:
                    assert float(b1[c, i]) ** 2 > float(b0[c, i]) ** 2
                else:
                    assert float(b1[c, i]) ** 2 < float(b0[c, i]) ** 2
    assert not np.any(a1[e] != a0[e]) and not np.any(a1[7] != a0[7])
