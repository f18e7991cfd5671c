"""Pins of the oracle's fl(.) operator (Def. 1-2, Table I) against independent
implementations: numpy's float32 cast and torch's bfloat16 / float16 /
float8_e4m3fn casts, plus the printed Table I parameters."""
import json
import os

import numpy as np
import pytest
import torch

from oracle.rounding import FORMATS, UNIT_ROUNDOFF, fl, pow2_scale, round_real

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def _values(seed=0, n=200_000):
    rng = np.random.default_rng(seed)
    parts = [
        rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n)),   # wide range
        rng.standard_normal(n),
        rng.uniform(-500, 500, n),
        np.ldexp(rng.integers(1, 2**12, n).astype(np.float64), rng.integers(-40, 20, n)),  # short significands: ties
        np.array([0.0, -0.0, np.inf, -np.inf, 448.0, 464.0, 465.0, 480.0, 65504.0, 65519.99, 65520.0,
                  2.0**-9, 2.0**-10, 3 * 2.0**-11, 2.0**-24, 2.0**-25, 2.0**-149, 2.0**-150, 1.5 * 2.0**-149,
                  3.3895313892515355e38, 3.4e38, 1e39]),
    ]
    v = np.concatenate(parts)
    return np.concatenate([v, -v])


@pytest.mark.parametrize("fmt,tdt", [("bf16", torch.bfloat16), ("fp16", torch.float16), ("e4m3", torch.float8_e4m3fn)])
def test_round_matches_torch_cast(fmt, tdt):
    # torch rounds float64 -> float32 -> target (two roundings); on float32-exact
    # inputs the first step is exact, so the casts are a single-rounding reference
    with np.errstate(over="ignore"):
        v = _values().astype(np.float32).astype(np.float64)
    if fmt == "e4m3":
        v = v[np.isfinite(v)]  # torch maps inf to nan as well; checked below
    ours = round_real(v, fmt)
    ref = torch.from_numpy(v).to(tdt).to(torch.float64).numpy()
    both_nan = np.isnan(ours) & np.isnan(ref)
    same = (ours == ref) & (np.signbit(ours) == np.signbit(ref))
    assert np.all(same | both_nan), v[~(same | both_nan)][:10]


def test_round_fp32_matches_numpy():
    v = _values(1)
    with np.errstate(over="ignore"):
        ref = v.astype(np.float32).astype(np.float64)
    ours = round_real(v, "fp32")
    assert np.array_equal(ours, ref, equal_nan=True)
    assert np.array_equal(np.signbit(ours), np.signbit(ref))


def test_e4m3_overflow_and_inf_are_nan():
    out = round_real(np.array([np.inf, -np.inf, 500.0, 464.0, -470.0]), "e4m3")
    assert np.isnan(out[0]) and np.isnan(out[1]) and np.isnan(out[2]) and np.isnan(out[4])
    assert out[3] == 448.0      # tie between 448 and 480 -> even significand -> 448


def test_complex_rounding_is_per_part():
    z = np.array([1 + 2.0**-9 + 1j * (1 + 3 * 2.0**-9)])
    out = fl(z, "bf16")
    assert out.real[0] == round_real(np.array([z.real[0]]), "bf16")[0]
    assert out.imag[0] == round_real(np.array([z.imag[0]]), "bf16")[0]


def test_table_I_parameters():
    t1 = GOLD["table_I"]
    for fmt in ("bf16", "fp16", "fp32"):
        row = t1[fmt]
        t, emin, xmax, _ = FORMATS[fmt]
        assert t == row["sig"]
        assert UNIT_ROUNDOFF[fmt] == pytest.approx(row["u"], rel=5e-3)
        assert 2.0**emin == pytest.approx(row["xmin"], rel=5e-3)
        assert xmax == pytest.approx(row["xmax"], rel=5e-3)
    # the printed fp64 u (4.88e-16) is a typo; 2^-53 is the unit roundoff of 53 significand bits
    assert UNIT_ROUNDOFF["fp64"] == pytest.approx(t1["fp64"]["u_correct"], rel=5e-3)
    assert UNIT_ROUNDOFF["fp64"] / t1["fp64"]["u_printed"] < 0.5


def test_standard_model_bound():
    """Def. 2: |fl(x) - x| <= u |x| for x in the normal range."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal(100_000) * 10
    for fmt in ("fp32", "bf16", "fp16", "e4m3"):
        xx = x[(np.abs(x) > 2.0 ** FORMATS[fmt][1]) & (np.abs(x) < FORMATS[fmt][2])]
        err = np.abs(round_real(xx, fmt) - xx)
        assert np.all(err <= UNIT_ROUNDOFF[fmt] * np.abs(xx) * (1 + 1e-12))
        assert np.max(err / np.abs(xx)) > 0.5 * UNIT_ROUNDOFF[fmt]   # the bound is attained


def test_pow2_scale():
    amax = np.array([1e-3, 0.7, 1.0, 448.0, 449.0, 3e4, 0.0, np.inf])
    s = pow2_scale(amax)
    fin = np.isfinite(amax) & (amax > 0)
    assert np.all(s[fin] * amax[fin] <= 448.0)
    assert np.all(2 * s[fin] * amax[fin] > 448.0)
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    assert s[6] == 1.0 and s[7] == 1.0


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "e4m3", "fp32"])
def test_round_is_nearest_on_float64_inputs(fmt):
    """fl(x) is representable and no representable neighbour is closer; ties even."""
    t, emin, xmax, _ = FORMATS[fmt]
    rng = np.random.default_rng(7)
    x = rng.standard_normal(50_000) * np.exp(rng.uniform(-8, 5, 50_000))
    x = x[np.abs(x) < xmax * 0.99]
    y = round_real(x, fmt)
    _, e2 = np.frexp(np.where(y == 0, 1.0, y))
    e = np.maximum(e2 - 1, emin)
    ulp = np.ldexp(1.0, e - (t - 1))
    k = y / ulp
    assert np.all(k == np.round(k))                      # representable
    lo, hi = y - ulp, y + ulp                            # neighbours (ulp below a binade edge is smaller: still a valid bracket)
    d = np.abs(y - x)
    assert np.all(d <= np.abs(lo - x)) and np.all(d <= np.abs(hi - x))
    tie = np.abs(d - ulp / 2) == 0
    assert np.all((k[tie] % 2) == 0)
