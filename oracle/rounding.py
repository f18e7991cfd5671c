"""The fl(.) operator of Def. 1 for the formats of Table I (plus fp8 e4m3fn).

A value is rounded to the nearest element of the target floating-point system
with ties to even (the IEEE default that Def. 2's standard model assumes),
keeping gradual underflow.  Table I gives the significand and exponent widths;
its fp64 unit roundoff is a typo (the correct value is 2^-53).

Formats: (t = significand bits including the hidden bit, emin = exponent of
the smallest normal number, xmax = largest finite value)
    fp32  t=24 emin=-126  xmax=(2-2^-23) 2^127   overflow -> inf
    bf16  t=8  emin=-126  xmax=(2-2^-7)  2^127   overflow -> inf
    fp16  t=11 emin=-14   xmax=65504             overflow -> inf
    e4m3  t=4  emin=-6    xmax=448               overflow -> nan (OCP "fn": no inf)
fp64 is the identity.

Test infrastructure only (see package docstring).
"""
from __future__ import annotations

import numpy as np

FORMATS = {
    #        t   emin   xmax                         overflow
    "fp32": (24, -126, (2.0 - 2.0**-23) * 2.0**127, "inf"),
    "bf16": (8, -126, (2.0 - 2.0**-7) * 2.0**127, "inf"),
    "fp16": (11, -14, 65504.0, "inf"),
    "e4m3": (4, -6, 448.0, "nan"),
}

# unit roundoff u = 2^-t (Table I, with the fp64 row corrected)
UNIT_ROUNDOFF = {"fp64": 2.0**-53, "fp32": 2.0**-24, "bf16": 2.0**-8, "fp16": 2.0**-11, "e4m3": 2.0**-4}


def round_real(x, fmt: str) -> np.ndarray:
    """Round a float64 array to ``fmt`` (RNE, gradual underflow); returns float64."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "fp64":
        return x.copy()
    t, emin, xmax, ovf = FORMATS[fmt]
    out = x.copy()
    fin = np.isfinite(x) & (x != 0.0)
    xf = x[fin]
    # exponent e with 2^e <= |x| < 2^(e+1); below the normal range the quantum is fixed
    _, e2 = np.frexp(xf)
    e = np.maximum(e2.astype(np.int64) - 1, emin)
    q = np.ldexp(1.0, (e - (t - 1)).astype(np.int64))
    y = np.rint(xf / q) * q              # x/q is exact (power-of-two scaling); rint ties to even
    big = np.abs(y) > xmax
    if np.any(big):
        y = y.copy()
        y[big] = np.copysign(np.inf, xf[big]) if ovf == "inf" else np.nan
    out[fin] = y
    if ovf == "nan":
        out[np.isinf(x)] = np.nan
    return out


def round_complex(z, fmt: str) -> np.ndarray:
    """Round real and imaginary parts separately (complex arithmetic on real units)."""
    z = np.asarray(z)
    if fmt == "fp64":
        return z.astype(np.complex128)
    return round_real(z.real, fmt) + 1j * round_real(z.imag, fmt)


def fl(z, fmt: str) -> np.ndarray:
    """fl(.) for real or complex arrays."""
    z = np.asarray(z)
    if np.iscomplexobj(z):
        return round_complex(z, fmt)
    return round_real(z, fmt)


def pow2_scale(amax, fmt: str = "e4m3") -> np.ndarray:
    """Power-of-two scale s = 2^floor(log2(xmax/amax)) that maps amax into range.

    Used for fp8 operands: multiplying by s is exact, and s*amax <= xmax so no
    value saturates.  amax == 0 or non-finite gives s = 1; the exponent is
    clamped to [-126, 126] so that s and 1/s are normal fp32 numbers.
    """
    amax = np.asarray(amax, dtype=np.float64)
    xmax = FORMATS[fmt][2]
    s = np.ones_like(amax)
    ok = np.isfinite(amax) & (amax > 0)
    ratio = xmax / amax[ok]
    _, e2 = np.frexp(ratio)            # ratio = m 2^e2, m in [0.5, 1) -> floor(log2) = e2 - 1
    s[ok] = np.ldexp(1.0, np.clip(e2.astype(np.int64) - 1, -126, 126))
    return s
