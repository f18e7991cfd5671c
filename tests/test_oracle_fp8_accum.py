"""Pins of the oracle's second rounding order for fp8 operands (the grouped,
truncating accumulation of `_trunc_group_sum` / `_seq_matmul_grouped`) and of
the R-conv reading (complex128 inputs reach the reduced operand formats
through fp32).

The grouped order is not taken from the paper: it is a model of how an fp8
matrix core adds a group of products (aligned to the largest product of the
group and truncated a fixed number of bits below it) and is used only as the
second of the two valid rounding orders whose distance measures how sensitive
an unconverged iterate is to the order of rounding.  These tests pin the code
to that stated definition with an independent element-by-element reference in
exact rational arithmetic (Fractions, one truncation per product, one
round-to-nearest-even per accumulator update), so that a slip in the
vectorised code (a wrong plane, sign, group boundary or exponent) fails here.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import detect as D
from oracle.rounding import round_real


def _fp32_rne(x: Fraction) -> Fraction:
    """Exact round-to-nearest-even of a rational to fp32 (normal and subnormal
    range; no overflow in these tests)."""
    if x == 0:
        return Fraction(0)
    sgn = -1 if x < 0 else 1
    a = abs(x)
    e = math.floor(math.log2(a.numerator) - math.log2(a.denominator))
    # fix the estimate: 2^e <= a < 2^(e+1)
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    q = Fraction(2) ** (e - 23)
    m = a / q
    fl_ = m.numerator // m.denominator
    rem = m - fl_
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl_ % 2 == 1):
        fl_ += 1
    return sgn * fl_ * q


def _trunc_ref(terms, frac_bits):
    """Definition: E = exponent of the largest |term| (2^E <= max < 2^(E+1));
    each term truncated toward zero to a multiple of 2^(E - frac_bits); the
    truncated terms added exactly."""
    fr = [Fraction(float(t)) for t in terms]
    mx = max(abs(t) for t in fr)
    if mx == 0:
        return Fraction(0)
    E = math.frexp(float(mx))[1] - 1
    q = Fraction(2) ** (E - frac_bits)
    tot = Fraction(0)
    for t in fr:
        k = t / q
        k_tr = math.trunc(k)            # toward zero
        tot += k_tr * q
    return tot


def _e4m3_values(rng, shape):
    """Random e4m3-representable values (products of two are exact in fp64)."""
    v = rng.standard_normal(shape) * np.exp(rng.uniform(-4, 4, shape))
    return round_real(np.clip(v, -448, 448), "e4m3")


def test_trunc_group_sum_special_cases():
    f = D._trunc_group_sum
    col = lambda *v: np.array(v, dtype=np.float64).reshape(-1, 1)
    # a product below the quantum 2^(E-13) is dropped, one at it is kept
    assert f(col(1.0, 2.0**-14), 13)[0] == 1.0
    assert f(col(1.0, 2.0**-13), 13)[0] == 1.0 + 2.0**-13
    # truncation is toward zero for negative products
    assert f(col(-1.0, -3 * 2.0**-14), 13)[0] == -1.0 - 2.0**-13
    assert f(col(1.0, -3 * 2.0**-14), 13)[0] == 1.0 - 2.0**-13
    # the largest product sets the exponent, whatever its sign or position
    assert f(col(2.0**-14, -1.5), 13)[0] == -1.5
    # all-zero group
    assert f(col(0.0, 0.0, -0.0), 13)[0] == 0.0
    # exactly representable groups come out exact
    assert f(col(1.0, 0.5, 0.25, 2.0**-13), 13)[0] == 1.75 + 2.0**-13


@pytest.mark.parametrize("seed", range(4))
def test_trunc_group_sum_matches_rational_reference(seed):
    rng = np.random.default_rng(seed)
    a = _e4m3_values(rng, (8, 60))
    b = _e4m3_values(rng, (8, 60))
    terms = a * b
    got = D._trunc_group_sum(terms, 13)
    for j in range(terms.shape[1]):
        ref = _trunc_ref(terms[:, j], 13)
        assert Fraction(float(got[j])) == ref, j
        # the truncation error is below one quantum per product
        exact = sum(Fraction(float(t)) for t in terms[:, j])
        mx = max(abs(float(t)) for t in terms[:, j])
        if mx > 0:
            q = 2.0 ** (math.frexp(mx)[1] - 1 - 13)
            assert abs(exact - ref) < 8 * Fraction(q)


@pytest.mark.parametrize("K,group", [(20, 8), (8, 8), (5, 8), (17, 4)])
def test_seq_matmul_grouped_matches_elementwise_reference(K, group):
    """Every output element, real plane and imaginary plane: groups of
    `group` consecutive contraction indices, in the order
        Re: (ar pr) group, then (-ai pi) group;  Im: (ai pr), then (ar pi)
    each group truncated-summed and added to the fp32 accumulator with one
    rounding, group after group."""
    rng = np.random.default_rng(K * 7 + group)
    A = _e4m3_values(rng, (1, 3, K)) + 1j * _e4m3_values(rng, (1, 3, K))
    P = _e4m3_values(rng, (1, K, 2)) + 1j * _e4m3_values(rng, (1, K, 2))
    got = D._seq_matmul_grouped(A, P, "fp32", group=group, frac_bits=13)
    for i in range(3):
        for c in range(2):
            wr = Fraction(0)
            wi = Fraction(0)
            for k0 in range(0, K, group):
                ks = range(k0, min(K, k0 + group))
                rr = [A[0, i, k].real * P[0, k, c].real for k in ks]
                ii = [-A[0, i, k].imag * P[0, k, c].imag for k in ks]
                ir = [A[0, i, k].imag * P[0, k, c].real for k in ks]
                ri = [A[0, i, k].real * P[0, k, c].imag for k in ks]
                wr = _fp32_rne(wr + _trunc_ref(rr, 13))
                wr = _fp32_rne(wr + _trunc_ref(ii, 13))
                wi = _fp32_rne(wi + _trunc_ref(ir, 13))
                wi = _fp32_rne(wi + _trunc_ref(ri, 13))
            assert Fraction(float(got[0, i, c].real)) == wr, (i, c)
            assert Fraction(float(got[0, i, c].imag)) == wi, (i, c)


def test_grouped_order_error_within_operand_rounding_bound():
    """The grouped order differs from the exact product by far less than the
    fp8 operand rounding the schedule already carries: per element at most
    (number of groups) x 8 quanta of 2^-13 relative to each group's largest
    product, plus the fp32 roundings (Thm 1 with u = 2^-24)."""
    rng = np.random.default_rng(3)
    K = 64
    A = _e4m3_values(rng, (2, 16, K)) + 1j * _e4m3_values(rng, (2, 16, K))
    P = _e4m3_values(rng, (2, K, 4)) + 1j * _e4m3_values(rng, (2, K, 4))
    got = D._seq_matmul_grouped(A, P, "fp32")
    ex = A @ P
    absprod = np.abs(A.real) @ np.abs(P.real) + np.abs(A.imag) @ np.abs(P.imag)
    absprod_i = np.abs(A.imag) @ np.abs(P.real) + np.abs(A.real) @ np.abs(P.imag)
    g = 2 * K / 8
    bound_r = absprod * (8 * 2.0**-13 + g * 2.0**-24 * 1.01)
    bound_i = absprod_i * (8 * 2.0**-13 + g * 2.0**-24 * 1.01)
    assert np.all(np.abs(got.real - ex.real) <= bound_r)
    assert np.all(np.abs(got.imag - ex.imag) <= bound_i)


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "e4m3"])
def test_r_conv_effect_is_rare_and_one_unit(fmt):
    """R-conv: a complex128 input is rounded to fp32 and then to the operand
    format; Def. 1 rounds once.  The two differ only where the fp32 value lands
    exactly on a midpoint of the operand format, which happens for about
    2^-(24 - t) of the values (t the format's significand bits), and then by
    one unit in the last place of the operand format."""
    rng = np.random.default_rng(11)
    n = 2_000_000
    v = rng.standard_normal(n) / np.sqrt(2 * 64)          # channel entries of CN(0, 1/64)
    if fmt == "e4m3":
        v = v * 448 / np.max(np.abs(v))
    once = round_real(v, fmt)
    twice = round_real(round_real(v, "fp32"), fmt)
    diff = once != twice
    t = {"fp16": 11, "bf16": 8, "e4m3": 4}[fmt]
    frac = diff.mean()
    assert frac <= 4 * 2.0 ** -(24 - t) + 10 / n
    if diff.any():
        _, e2 = np.frexp(once[diff])
        ulp = np.ldexp(1.0, e2 - t)
        assert np.all(np.abs(once[diff] - twice[diff]) <= ulp * (1 + 1e-12))
