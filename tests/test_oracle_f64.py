"""Pins of the oracle's binary64 variant (the paper's precision, Sec. V)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pi(digits):
    """pi to `digits` decimals by Machin's formula, pi = 16 atan(1/5) - 4 atan(1/239),
    in integer fixed point (truncation error below 10^-(digits - 5))."""
    scale = 10 ** (digits + 10)

    def atan_inv(n):
        term = scale // n
        total, k, sign = 0, 1, 1
        while term:
            total += sign * (term // k)
            term //= n * n
            k += 2
            sign = -sign
        return total

    return Fraction(16 * atan_inv(5) - 4 * atan_inv(239), scale)


def _cos_sin(x, terms=40):
    """cos x and sin x by their Taylor series, exactly in rationals (|x| < 0.1:
    the first omitted term is below 10^-100)."""
    c, s_, term = Fraction(0), Fraction(0), Fraction(1)
    for k in range(2 * terms):
        if k % 2 == 0:
            c += term if (k // 2) % 2 == 0 else -term
        else:
            s_ += term if (k // 2) % 2 == 0 else -term
        term = term * x / (k + 1)
    return c, s_


def _correctly_rounded(value, x, precision_bits, margin=Fraction(1, 10 ** 80)):
    """x is the float of `precision_bits` significand bits nearest `value`
    (strictly within half an ulp, by more than the error of `value`)."""
    _, e = math.frexp(x)                    # x = m 2^e, 0.5 <= m < 1
    half_ulp = Fraction(2) ** (e - precision_bits - 1)
    return abs(Fraction(x) - value) + margin < half_ulp


def test_gate_constants_are_the_correctly_rounded_values():
    """The oracle's rotation constants, binary32 and binary64, are the values
    of cos(pi/100), sin(pi/100) and 1/sqrt(2) rounded to nearest in their
    precision, checked against 90-digit values of the functions (pi from
    Machin's formula, cos and sin from their Taylor series, 1/sqrt(2) by
    squaring): a half-ulp test with rationals, no libm involved."""
    import re
    src = open(os.path.join(ROOT, "oracle", "qieo_oracle.c")).read()
    const = dict(re.findall(r"#define (ROT_C|ROT_S|AMP0|ROT_C64|ROT_S64|AMP0_64)\s+(\S+)", src))
    assert set(const) == {"ROT_C", "ROT_S", "AMP0", "ROT_C64", "ROT_S64", "AMP0_64"}
    f32 = {k: float.fromhex(v.rstrip("f")) for k, v in const.items() if not k.endswith("64")}
    f64 = {k[:-3] if k.endswith("_64") else k[:-2]: float.fromhex(v)
           for k, v in const.items() if k.endswith("64")}
    for v in f32.values():                   # exactly representable in binary32
        assert float(np.float32(v)) == v
    c, s_ = _cos_sin(_pi(90) / 100)
    assert abs(c * c + s_ * s_ - 1) < Fraction(1, 10 ** 85)
    for name, x, bits in (("cos", f32["ROT_C"], 24), ("sin", f32["ROT_S"], 24),
                          ("cos", f64["ROT_C"], 53), ("sin", f64["ROT_S"], 53)):
        assert _correctly_rounded(c if name == "cos" else s_, x, bits), (name, bits, x.hex())
    # 1/sqrt(2): x is the nearest float iff (x -+ half ulp)^2 bracket 1/2
    for x, bits in ((f32["AMP0"], 24), (f64["AMP0"], 53)):
        _, e = math.frexp(x)
        h = Fraction(2) ** (e - bits - 1)
        assert (Fraction(x) - h) ** 2 < Fraction(1, 2) < (Fraction(x) + h) ** 2, bits
    # the constants move angles by 0.01 pi: atan2(S, C) within an ulp of pi/100
    assert abs(math.atan2(f64["ROT_S"], f64["ROT_C"]) - math.pi / 100) < 1e-17


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
