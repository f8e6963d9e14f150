"""Pins of the exact Python references (oracle/exact.py) against IEEE square roots and closed forms."""
import math
import random
from fractions import Fraction

import numpy as np

from oracle import exact


def test_rn_sqrt_matches_ieee_sqrt_f64():
    rng = random.Random(1)
    for _ in range(20000):
        x = math.ldexp(rng.randrange(1, 1 << 53), rng.randrange(-1126, 970))
        if x == 0 or math.isinf(x):
            continue
        fr = Fraction(x)
        N, E = exact._dyadic(fr)
        assert exact.rn_sqrt_dyadic(N, E, "f64") == math.sqrt(x)


def test_rn_sqrt_matches_ieee_sqrt_f32():
    rng = np.random.default_rng(2)
    bits = rng.integers(1, 0x7F800000, size=20000, dtype=np.uint32)
    xs = bits.view(np.float32)
    ref = np.sqrt(xs)
    for x, r in zip(xs.tolist(), ref.tolist()):
        N, E = exact._dyadic(Fraction(x))
        assert exact.rn_sqrt_dyadic(N, E, "f32") == r


def test_pythagorean_and_scaled():
    for a, b, c in [(3, 4, 5), (5, 12, 13), (8, 15, 17), (20, 21, 29), (119, 120, 169)]:
        for k in (-1074, -1070, -600, -30, 0, 30, 900):
            x, y = math.ldexp(a, k), math.ldexp(b, k)
            if math.ldexp(c, k) > 1.7976931348623157e308:
                continue
            assert exact.cr_hypot_exact(x, y) == math.ldexp(c, k)
    assert exact.cr_hypot_exact(3 * 2.0 ** -149, 4 * 2.0 ** -149, "f32") == 5 * 2.0 ** -149


def test_subnormal_and_overflow_rounding():
    tiny = 2.0 ** -1074
    # sqrt(2) * 2^-1074 rounds to 2^-1074 on the subnormal grid
    assert exact.cr_hypot_exact(tiny, tiny) == tiny
    # sqrt(5) 2^-1074 ~ 2.236 -> 2
    assert exact.cr_hypot_exact(2 * tiny, tiny) == 2 * tiny
    big = 1.7976931348623157e308
    assert exact.cr_hypot_exact(big, big) == math.inf
    assert exact.cr_hypot_exact(big, 1.0) == big
    r = exact.cr_hypot_exact(big / 2, big / 2)
    assert r == float(np.float64(big / 2) * np.sqrt(2.0)) or abs(r / (big / math.sqrt(2)) - 1) < 2e-16
    # overflow threshold: DBL_MAX + ulp/2 rounds to even -> inf; just below stays finite
    half_ulp = 2.0 ** 970
    N = (int(big) + int(half_ulp)) ** 2
    assert exact.rn_sqrt_dyadic(N, 0) == math.inf
    assert exact.rn_sqrt_dyadic(N - 1, 0) == big


def test_ties_round_to_even():
    # C = 2^53 + 1 is a midpoint between 2^53 and 2^53 + 2; C^2 = N exactly -> tie -> even (2^53).
    C = (1 << 53) + 1
    assert exact.rn_sqrt_dyadic(C * C, 0) == float(1 << 53)
    C = (1 << 53) + 3  # midpoint between 2^53 + 2 (mantissa odd) and 2^53 + 4 (even)
    assert exact.rn_sqrt_dyadic(C * C, 0) == float((1 << 53) + 4)
    assert exact.rn_sqrt_dyadic(C * C - 1, 0) == float((1 << 53) + 2)
    assert exact.rn_sqrt_dyadic(C * C + 1, 0) == float((1 << 53) + 4)


def test_R_exact_small_cases():
    assert exact.R_exact_A([3.0]) == 3.0
    assert exact.R_exact_A([-3.0, 4.0]) == 5.0
    assert exact.R_exact_A([1.0, 2.0, 2.0]) == exact.cr_hypot_exact(exact.cr_hypot_exact(1.0, 2.0), 2.0)
    assert exact.nrm2_exact([1.0, 2.0, 2.0]) == 3.0
