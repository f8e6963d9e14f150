"""Pins of the oracle's node functions: cr_hypot[f] (exact big-integer rounding), v1_hypot
(Listing 2 properties and the Eq. (reH) bound), cr_pow (mpmath), v1_lp (Listing 5 / Eq. (sp))."""
import math
import random
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from oracle import bounds, exact

F32MAX = float(np.finfo(np.float32).max)


def _pairs_f64(rng, count):
    out = []
    for _ in range(count):
        kind = rng.random()
        ea = rng.randrange(-1100, 1024)
        a = math.ldexp(rng.random() + 0.5, ea)
        if kind < 0.4:
            b = math.ldexp(rng.random() + 0.5, ea + rng.randrange(-30, 1))
        elif kind < 0.6:
            b = math.ldexp(rng.random() + 0.5, ea + rng.randrange(-80, 5))
        elif kind < 0.8:
            b = a * (1 + rng.random() * 1e-3)
        else:
            b = math.ldexp(rng.random(), rng.randrange(-1080, 1024))
        if math.isinf(a) or math.isinf(b):
            continue
        out.append((a, b))
    return out


def test_cr_hypot_matches_exact_random():
    rng = random.Random(11)
    for a, b in _pairs_f64(rng, 30000):
        assert oracle.cr_hypot(a, b) == exact.cr_hypot_exact(a, b), (a, b)
    assert oracle.counters()["exact_failures"] == 0


def _euclid_ties(bits, count, rng):
    """Pythagorean triples (A, B, C) with C odd in [2^bits, 2^(bits+1)), A, B < 2^bits: sqrt is a midpoint."""
    out = []
    t = 1 + math.sqrt(2)
    while len(out) < count:
        v = int(math.sqrt(rng.uniform(1.02, 1.38) * 2 ** bits / (t * t + 1)))
        u = int(v * rng.uniform(2.2, 2.6))
        if (u - v) % 2 == 0 or math.gcd(u, v) != 1:
            continue
        A, B, C = u * u - v * v, 2 * u * v, u * u + v * v
        if A < 2 ** bits and B < 2 ** bits and 2 ** bits <= C < 2 ** (bits + 1):
            out.append((A, B, C))
    return out


def test_cr_hypot_exact_ties_and_near_ties():
    rng = random.Random(3)
    for A, B, C in _euclid_ties(53, 300, rng):
        for k in (-1074, -600, 0, 500, 916):
            a, b = math.ldexp(A, k), math.ldexp(B, k)
            want = exact.cr_hypot_exact(a, b)
            assert oracle.cr_hypot(a, b) == want
            # the exact tie goes to the even neighbour of C 2^k
            if k == 0:
                assert want in (float(C - 1), float(C + 1)) and (int(want) // 2) % 2 == 0
            a2 = math.nextafter(a, math.inf)
            assert oracle.cr_hypot(a2, b) == exact.cr_hypot_exact(a2, b)
            b2 = math.nextafter(b, 0)
            assert oracle.cr_hypot(a, b2) == exact.cr_hypot_exact(a, b2)


def test_cr_hypotf_matches_exact():
    rng = random.Random(5)
    for _ in range(30000):
        ea = rng.randrange(-150, 128)
        a = float(np.float32(math.ldexp(rng.random() + 0.5, ea)))
        b = float(np.float32(math.ldexp(rng.random() + 0.5, min(ea + rng.randrange(-20, 1), 127))))
        if math.isinf(a) or math.isinf(b):
            continue
        assert oracle.cr_hypotf(a, b) == exact.cr_hypot_exact(a, b, "f32"), (a, b)
    for A, B, C in _euclid_ties(24, 200, rng):
        for k in (-149, -60, 0, 80):
            a, b = math.ldexp(A, k), math.ldexp(B, k)
            assert oracle.cr_hypotf(a, b) == exact.cr_hypot_exact(a, b, "f32")


def test_cr_hypot_closed_forms():
    tiny = 2.0 ** -1074
    big = 1.7976931348623157e308
    assert oracle.cr_hypot(3.0, 4.0) == 5.0
    assert oracle.cr_hypot(-5.0, 12.0) == 13.0
    assert oracle.cr_hypot(3 * tiny, 4 * tiny) == 5 * tiny
    assert oracle.cr_hypot(big, big) == math.inf
    assert oracle.cr_hypot(big, tiny) == big
    assert oracle.cr_hypot(big / 2, big / 2) == exact.cr_hypot_exact(big / 2, big / 2) < math.inf
    assert oracle.cr_hypot(0.0, 0.0) == 0.0
    assert oracle.cr_hypot(math.inf, math.nan) == math.inf
    assert math.isnan(oracle.cr_hypot(math.nan, 1.0))
    assert oracle.cr_hypotf(F32MAX, F32MAX) == math.inf
    assert oracle.cr_hypotf(3 * 2.0 ** -149, 4 * 2.0 ** -149) == 5 * 2.0 ** -149


def _rel_bound_ok(h, a, b, factor):
    """|h - sqrt(a^2+b^2)| <= (factor - 1) sqrt(a^2+b^2), checked exactly via squares."""
    S = Fraction(a) ** 2 + Fraction(b) ** 2
    f = Fraction(factor)
    lo, hi = (2 - f), f
    H = Fraction(h) ** 2
    return lo * lo * S <= H <= hi * hi * S


def test_v1_hypot_properties_and_bound():
    fac = bounds.node_factor("v1", "f64")
    fac = Fraction(str(mpmath.nstr(fac, 40)))
    assert oracle.v1_hypot(3.0, 4.0) == 5.0
    assert oracle.v1_hypot(0.0, 0.0) == 0.0
    rng = random.Random(7)
    for a, b in _pairs_f64(rng, 5000):
        if a > 1e300 or b > 1e300 or a < 1e-300 or b < 1e-300:
            continue
        h = oracle.v1_hypot(a, b)
        assert h == oracle.v1_hypot(b, a) == oracle.v1_hypot(-a, b)
        assert oracle.v1_hypot(a, 0.0) == a
        assert _rel_bound_ok(h, a, b, fac)


def test_v1_hypot_does_not_propagate_nan():
    # Listing 2's closing comment: fmin / fmax return the other argument if one is a NaN,
    # so both m and M become that argument and no NaN comes out.
    assert oracle.v1_hypot(math.nan, 3.0) == oracle.v1_hypot(3.0, 3.0)


def _nearest_check(c, ref_mp, nxt):
    up, dn = nxt(c, math.inf), nxt(c, 0.0)
    d0 = abs(mpmath.mpf(c) - ref_mp)
    return d0 <= abs(mpmath.mpf(up) - ref_mp) and d0 <= abs(mpmath.mpf(dn) - ref_mp)


def test_cr_pow_is_nearest_against_mpmath():
    mpmath.mp.prec = 300
    rng = random.Random(13)
    for _ in range(3000):
        if rng.random() < 0.5:
            x, y = rng.random(), rng.choice([0.75, 1.5, 2.25, 4.0, 0.5 * math.pi, 0.7071067811865476, 1.25])
        else:
            x, y = 1 + rng.random(), 1.0 / rng.choice([1.5, 3.0, 4.5, 8.0, math.e, math.sqrt(2), 0.5])
        c = oracle.cr_pow(x, y)
        assert _nearest_check(c, mpmath.power(mpmath.mpf(x), mpmath.mpf(y)), math.nextafter)
        cf = oracle.cr_powf(float(np.float32(x)), float(np.float32(y)))
        ref = mpmath.power(mpmath.mpf(float(np.float32(x))), mpmath.mpf(float(np.float32(y))))
        f32next = lambda v, d: float(np.nextafter(np.float32(v), np.float32(d)))  # noqa: E731
        assert _nearest_check(cf, ref, f32next)
    assert oracle.counters()["pow_unresolved"] == 0


def test_powq_accuracy_against_mpmath():
    # the Ziv margin in cr_pow assumes powq is accurate to ~2^-104 relative
    mpmath.mp.prec = 300
    rng = random.Random(17)
    worst = 0
    for _ in range(2000):
        x, y = rng.random() * 2, rng.random() * 5
        hi, lo = oracle.powq(x, y)
        ref = mpmath.power(mpmath.mpf(x), mpmath.mpf(y))
        if ref == 0:
            continue
        err = abs((mpmath.mpf(hi) + mpmath.mpf(lo) - ref) / ref)
        worst = max(worst, float(err))
    assert worst < 2.0 ** -104


def test_p_cutoff_of_section_4():
    # Sect. 4: with cr_pow, pow(z, RN(1/p')) = 1 for all z in [1, 2] first happens for 2^52 < p' <= 2^53.
    assert oracle.cr_pow(2.0, 2.0 ** -53) == 1.0
    assert oracle.cr_pow(1.5, 2.0 ** -53) == 1.0
    assert oracle.cr_pow(2.0, 2.0 ** -52) > 1.0
    # ... and with cr_powf, 2^23 < p' <= 2^24.
    assert oracle.cr_powf(2.0, 2.0 ** -24) == 1.0
    assert oracle.cr_powf(2.0, 2.0 ** -23) > 1.0


def test_v1_lp_reduces_to_v1_hypot_at_p2():
    # Eq. (sp): with p = 2 the p-node is exactly v1_hypot (pow(Q, 1) = Q, pow(Z, 1/2) = sqrt(Z)).
    rng = random.Random(19)
    for a, b in _pairs_f64(rng, 3000):
        if a > 1e300 or b > 1e300:
            continue
        assert oracle.v1_lp(2.0, a, b) == oracle.v1_hypot(a, b)
    for _ in range(2000):
        a, b = float(np.float32(rng.random())), float(np.float32(rng.random() * 100))
        assert oracle.v1_lpf(2.0, a, b) == oracle.v1_hypotf(a, b)


def test_v1_lp_closed_forms():
    # (|x|^p + |y|^p)^(1/p) for exactly representable cases
    assert oracle.v1_lp(3.0, 0.0, 5.0) == 5.0
    assert oracle.v1_lp(4.0, 1.0, 1.0) == oracle.cr_pow(2.0, 0.25)
    assert oracle.v1_lp(8.0, 2.0, 2.0) == 2.0 * oracle.cr_pow(2.0, 0.125)
    assert oracle.v1_lp(0.5, 1.0, 1.0) == 4.0  # quasi-norm: (1 + 1)^2
    for p in (1.5, 3.0, 4.5, 8.0):
        r = oracle.v1_lp(p, 3.0, 4.0)
        mpmath.mp.prec = 200
        ref = mpmath.power(mpmath.power(3, p) + mpmath.power(4, p), 1 / mpmath.mpf(p))
        assert abs(r - float(ref)) <= 4 * 2.0 ** -53 * float(ref)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_sum_and_max_nodes_via_recursion(fmt):
    dt = np.float64 if fmt == "f64" else np.float32
    x = np.array([1, -2, 3, -4, 5, 6, -7], dtype=dt)
    assert oracle.nrmp(x, 1.0) == 28
    assert oracle.nrmp(x, math.inf) == 7
    assert oracle.nrmp(x, 2.0 ** 60) == 7


def test_cr_pow_hard_case_goes_to_mpfr():
    # (1 + 4 ulp)^(1/8) lies about 2^-104 below the midpoint 1 + 2^-53: binary128 alone is borderline.
    z = 1.0 + 4 * 2.0 ** -52
    mpmath.mp.prec = 400
    assert _nearest_check(oracle.cr_pow(z, 0.125), mpmath.power(mpmath.mpf(z), mpmath.mpf(0.125)),
                          math.nextafter)
    assert oracle.cr_pow(z, 0.125) == oracle.mpfr_pow(z, 0.125)
    rng = random.Random(23)
    for _ in range(500):
        x, y = rng.random() * 2, rng.choice([0.25, 0.125, 2.0 / 3.0, 1.0 / 3.0, 0.75, 2.25, 4.0])
        assert oracle.cr_pow(x, y) == oracle.mpfr_pow(x, y)
        assert oracle.cr_powf(x, y) == np.float32(oracle.mpfr_pow(float(np.float32(x)), float(np.float32(y)), 24))
    assert oracle.counters()["pow_unresolved"] == 0


def test_pnorm_recursion_reference_closed_forms():
    """With exactly representable p/2 and 1/p (p = 4, 1/2, 1) the binary128 recursion equals
    the flat binary128 p-norm; for p = 2 it is the exact Frobenius norm to binary128."""
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, 3001)
    for p in (4.0, 0.5, 1.0, 2.0):
        hi, lo = oracle.ref_pnorm_R(x, p)
        fh, fl = oracle.ref_pnorm(x, p)
        assert abs((hi + lo) - (fh + fl)) <= 1e-28 * (fh + fl), p
    hi, lo = oracle.ref_pnorm_R(x, 2.0)
    assert hi == oracle.exact_nrm2(x)


def test_pnorm_recursion_reference_keeps_the_exponent_rounding():
    """For p = RN(2/3), RN(1/p) = 1.5 is not 1/p: the recursion with the method's exponents
    differs from the flat p-norm by a bias that grows with the depth of the tree."""
    x = np.full(1 << 12, 0.5)
    p = 2.0 / 3.0
    hi, lo = oracle.ref_pnorm_R(x, p)
    fh, fl = oracle.ref_pnorm(x, p)
    rel = abs((hi + lo) - (fh + fl)) / (fh + fl)
    assert 2 * 2.0 ** -53 < rel < 20 * 2.0 ** -53
