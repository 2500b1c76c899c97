"""The error bound of the int8 Ozaki split, checked on the CPU (no GPU).

The GPU tests hold the Ozaki forwards to (S + 1.05) 2^-7S K 2^(e_i + e_j)
per Gram entry.  Here the split is carried out as defined (x = w 2^(6 - e),
|x| < 64; S times d = rint(x) in FP32, x = (x - d) 128), every product of
two elements is rebuilt from the kept levels s + t < S exactly (fractions),
and its error is compared with the per-product bound (S + 1.05) 2^-7S
2^(e_i + e_j), for S = 4, 5, 6, on elements spread over many binades and on
worst-case-like values just below a power of two.  Also: the digits stay
within |d| <= 64, and a level sum of S products of K = 87,381 terms (the
library's limit) stays below 2^31.
"""
from fractions import Fraction

import numpy as np
import pytest


def split(w, S):
    """Digits of FP32 value w (row exponent from w itself): list of ints, e."""
    m = abs(float(w))
    e = int(np.frexp(np.float32(m))[1]) if m > 0 else 0
    x = np.float32(np.ldexp(np.float32(w), 6 - e))
    digits = []
    for _ in range(S):
        d = np.float32(np.rint(x))
        digits.append(int(d))
        x = np.float32((x - d) * np.float32(128.0))
    return digits, e


def product_error(a, b, S):
    da, ea = split(a, S)
    db, eb = split(b, S)
    approx = Fraction(0)
    for s in range(S):
        for t in range(S - s):       # levels s + t < S
            approx += Fraction(da[s] * db[t]) / Fraction(2) ** (7 * (s + t))
    approx *= Fraction(2) ** (ea - 6) * Fraction(2) ** (eb - 6)
    exact = Fraction(float(np.float32(a))) * Fraction(float(np.float32(b)))
    return abs(exact - approx), Fraction(2) ** (ea + eb), da + db


@pytest.mark.parametrize("S", [4, 5, 6])
def test_per_product_error_within_bound(S):
    rng = np.random.default_rng(17 + S)
    vals = np.concatenate([
        rng.standard_normal(300) * np.ldexp(1.0, rng.integers(-40, 40, 300)),
        np.nextafter(np.float32(np.ldexp(1.0, rng.integers(-20, 20, 40))), np.float32(0)),  # just below 2^e
        np.ldexp(1.0, rng.integers(-20, 20, 20)),                                         # exact powers of two
    ]).astype(np.float32)
    worst = Fraction(0)
    for q in range(0, len(vals) - 1):
        err, scale, digits = product_error(vals[q], vals[q + 1], S)
        assert max(abs(d) for d in digits) <= 64
        worst = max(worst, err / scale)
    bound = Fraction(S * 100 + 105, 100) / Fraction(2) ** (7 * S)
    assert worst <= bound, (S, float(worst), float(bound))


def test_level_sums_stay_exact_in_int32():
    k_max = ((1 << 31) - 1) // (6 * 64 * 64)   # the library's K limit for the Ozaki forward (87,381)
    for S in (4, 5, 6):
        assert S * k_max * 64 * 64 < 2 ** 31
