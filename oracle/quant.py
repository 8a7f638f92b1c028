"""FP8 (E4M3) quantization of a factor for FP8 x FP8 first contractions, in
FP64 NumPy.  Not from the paper (it computes in FP64): the reading of the
precision path in which both operands of the first contraction are E4M3.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The format (OCP 8-bit floating point, variant E4M3 "fn"): a sign bit, four
exponent bits with bias 7 and three mantissa bits; exponent field 0 holds the
subnormals m * 2^-9, field e > 0 the normals (1 + m/8) * 2^(e-7); the code
with all exponent and mantissa bits set is NaN and there are no infinities,
so the largest finite magnitude is 448.

Pins (tests marked "not gpu", tests/test_oracle_quant.py):
  e4m3_values        -> count, spacing and extremes fixed by the format
                        (127 non-negative finite values, 2^-9 .. 448)
  e4m3_round         -> every finite value maps to itself; midpoints between
                        neighbours go to the even code; against torch's own
                        float8_e4m3fn conversion on random and boundary inputs
  quantize_columns   -> the scaled column maximum lies in (224, 448], the
                        scale is a power of two, and the dequantized factor
                        is within half an E4M3 step of each entry
"""

import numpy as np


def e4m3_values():
    """The non-negative finite E4M3 values in code order (codes 0x00 .. 0x7E),
    from the format's definition: exponent field e, mantissa m."""
    vals = []
    for code in range(0x7F):
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals, dtype=np.float64)


_VALS = e4m3_values()


def e4m3_round(x):
    """Round each |x| <= 448 to the nearest E4M3 value, a tie going to the
    value whose code is even (the one with an even mantissa); the sign is
    kept.  Returns FP64 values."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    if a.size and np.max(a) > 448.0:
        raise ValueError("e4m3_round: magnitude beyond 448")
    hi = np.searchsorted(_VALS, a, side="left")  # first value >= a
    hi = np.minimum(hi, len(_VALS) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _VALS[lo]
    dhi = _VALS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    return np.sign(x) * _VALS[code]


def quantize_columns(A):
    """Column-wise E4M3 quantization of a factor A (s x R): column c is
    multiplied by 2^e_c, the largest power of two for which its largest
    magnitude stays at or below 448 (e_c clamped to [-120, 120]; 0 for a zero
    column), rounded by e4m3_round, and divided by 2^e_c again.  Returns the
    dequantized factor (FP64) and the exponents e_c.  The input is taken as
    given (the contraction quantizes the FP32 copy of a factor, so callers
    pass that copy)."""
    A = np.asarray(A, dtype=np.float64)
    out = np.empty_like(A)
    exps = np.zeros(A.shape[1], dtype=np.int64)
    for c in range(A.shape[1]):
        col = A[:, c]
        mx = float(np.max(np.abs(col))) if col.size else 0.0
        e = 0
        if mx > 0.0:
            e = int(np.floor(np.log2(448.0 / mx)))
            while mx * 2.0 ** e > 448.0:  # the logarithm's rounding, either way
                e -= 1
            while mx * 2.0 ** (e + 1) <= 448.0:
                e += 1
            e = min(max(e, -120), 120)
        exps[c] = e
        out[:, c] = e4m3_round(col * 2.0 ** e) * 2.0 ** (-e)
    return out, exps
