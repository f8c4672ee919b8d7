"""Pins of the oracle's binary64 variant (the paper's precision, Sec. V)."""
import math

import numpy as np
import pytest

import workloads


def test_binary64_constants_are_the_correctly_rounded_values(oracle_mod):
    # correctly rounded binary64 values of cos(pi/100), sin(pi/100), 1/sqrt(2)
    # (computed to 60 digits with Machin's pi and Taylor series); libm agrees
    # on the first two
    assert float.fromhex("0x1.ffbf52e9d1086p-1") == math.cos(0.01 * math.pi)
    assert float.fromhex("0x1.015122df75860p-5") == math.sin(0.01 * math.pi)
    from fractions import Fraction
    x = Fraction(float.fromhex("0x1.6a09e667f3bcdp-1"))
    half_ulp = Fraction(1, 2 ** 54)            # ulp of [0.5, 1) is 2^-53
    assert (x - half_ulp) ** 2 < Fraction(1, 2) < (x + half_ulp) ** 2


def test_f64_closed_form_angle_tracking(oracle_mod):
    phi = math.atan2(float.fromhex("0x1.015122df75860p-5"), float.fromhex("0x1.ffbf52e9d1086p-1"))
    a = b = float.fromhex("0x1.6a09e667f3bcdp-1")
    for k in range(1, 25):
        a, b, rot = oracle_mod.cip_gene_f64(a, b, 1)
        assert rot
        assert abs(a - math.cos(math.pi / 4 + k * phi)) < 1e-15 * k + 1e-16
        assert abs(b - math.sin(math.pi / 4 + k * phi)) < 1e-15 * k + 1e-16


@pytest.mark.parametrize("deg", [20, 110, 200, 290])
def test_f64_moves_toward_target_in_every_quadrant(oracle_mod, deg):
    th = math.radians(deg)
    a, b = math.cos(th), math.sin(th)
    assert oracle_mod.cip_gene_f64(a, b, 1)[1] ** 2 > b ** 2
    assert oracle_mod.cip_gene_f64(a, b, 0)[1] ** 2 < b ** 2


def test_f64_norm_and_quality(oracle_mod):
    inst = workloads.small_instance()
    o = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                          precision=64)
    worst = 0.0
    for _ in range(inst.generations):
        o.generation()
        a, b = o.amplitudes()
        worst = max(worst, float(np.abs(a * a + b * b - 1).max()))
    assert worst < 1e-14
    opt = oracle_mod.knap_dp(inst.values, inst.weights, inst.capacity)
    assert 0.8 * opt < o.best().fitness <= opt


def test_f64_first_generation_equals_f32_observation(oracle_mod):
    """Generation 0 observes fl(1/sqrt2)^2 in each precision against the same
    24-bit draws; both squares lie within 2^-24 of 1/2 and no draw is exactly
    1/2 +- tiny, so the first alleles agree."""
    inst = workloads.random_instance(500, 20, seed=3)
    o32 = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed)
    o64 = oracle_mod.Oracle(inst.values, inst.weights, inst.capacity, inst.n_pop, inst.seed,
                            precision=64)
    o32.generation()
    o64.generation()
    assert np.array_equal(o32.alleles(), o64.alleles())
    assert o32.elite == o64.elite
