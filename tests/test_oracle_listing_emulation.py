"""Bitwise pins of the oracle's Listing 2 and Listing 5 nodes by an exact emulation.

Each statement of Listing 2 (v1_hypot) and Listing 5 (v1_lp, Eq. (qp)) is one IEEE
operation; here every one is evaluated exactly in rational arithmetic and rounded once to
nearest-even in the working format (binary64 for D, binary32 for S), with subnormal results
and overflow to infinity:

  X = |x|, Y = |y|, m = fmin(X, Y), M = fmax(X, Y), q = RN(m / M), Q = fmax(q, 0)
  Listing 2:  S = RN(Q^2 + 1) (one fma), s = RN(sqrt(S)), result RN(M s)
  Listing 5:  S = RN(Q^RN(p/2)), Z = RN(S^2 + 1) (one fma), C = RN(Z^RN(1/p)), RN(M C)

with RN(p/2) and RN(1/p) rounded once in the working format (Sect. 4: the exponents are
computed once, 1/p rounded; single precision replaces double throughout, Sect. 2).  The
powers are correctly rounded: an exact root where x^y is rational (y with a denominator of
at most 2^8 and x a perfect power), otherwise mpmath at 400 bits with a rounding-boundary
check.  Nothing here calls the oracle's arithmetic; the oracle's results must equal these
bit for bit.
"""
import math
import random
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from oracle import exact

FMTS = {"f64": (53, -1074, 1024), "f32": (24, -149, 128)}
INF = math.inf


def rn(v, fmt):
    """v (a Fraction >= 0, or +inf) rounded to nearest-even in fmt; +inf on overflow."""
    if v == INF:
        return INF
    if v == 0:
        return 0.0
    prec, ulp_min, emax = FMTS[fmt]
    num, den = v.numerator, v.denominator
    e = num.bit_length() - den.bit_length()  # 2^e <= v < 2^(e+2)
    if Fraction(num, den) < Fraction(2) ** e:
        e -= 1
    if Fraction(num, den) >= Fraction(2) ** (e + 1):
        e += 1
    k = max(e - (prec - 1), ulp_min)  # exponent of the result's ulp
    s = v / Fraction(2) ** k
    q, r = divmod(s.numerator, s.denominator)
    twice = 2 * r
    if twice > s.denominator or (twice == s.denominator and q & 1):
        q += 1
    if q.bit_length() + k > emax:  # q 2^k >= 2^emax
        return INF
    return math.ldexp(q, k)


def F(x):
    return Fraction(x)


def div(a, b, fmt):
    """IEEE a / b for a, b >= 0: 0/0 and inf/inf are NaN, a/0 is inf, finite/inf is 0."""
    if (a == 0 and b == 0) or (a == INF and b == INF):
        return math.nan
    if b == 0 or a == INF:
        return INF
    if b == INF:
        return 0.0
    return rn(F(a) / F(b), fmt)


def mul(a, b, fmt):
    if a == INF or b == INF:
        return math.nan if (a == 0 or b == 0) else INF
    return rn(F(a) * F(b), fmt)


def fma_sq1(a, fmt):
    """RN(a a + 1), one rounding."""
    return INF if a == INF else rn(F(a) * F(a) + 1, fmt)


def fmax(a, b):
    """IEEE maxNum: a NaN operand gives the other one."""
    if a != a:
        return b
    if b != b:
        return a
    return a if a >= b else b


def fmin(a, b):
    if a != a:
        return b
    if b != b:
        return a
    return a if a <= b else b


def sqrt_rn(a, fmt):
    if a == INF or a == 0:
        return a
    f = F(a)
    N, D = f.numerator, f.denominator  # D is a power of two
    return exact.rn_sqrt_dyadic(N, -(D.bit_length() - 1), fmt)


def _exact_root(f, k):
    """f^(1/2^k) if it is a dyadic rational, else None (f > 0 dyadic)."""
    N, D = f.numerator, f.denominator
    E = D.bit_length() - 1
    r = 1 << k
    if E % r:
        return None
    root = N
    for _ in range(k):
        s = math.isqrt(root)
        if s * s != root:
            return None
        root = s
    return Fraction(root, 1 << (E // r))


def _ambiguous(v, fmt):
    """v (mpf) within 2^-380 (relative) of a rounding boundary of fmt."""
    prec, ulp_min, _ = FMTS[fmt]
    man, ex = v.man, v.exp
    f = Fraction(int(man)) * Fraction(2) ** int(ex)
    e = math.floor(mpmath.log(v, 2))
    k = max(e - (prec - 1), ulp_min)
    s = f / Fraction(2) ** k
    frac = s - (s.numerator // s.denominator)
    return abs(frac - Fraction(1, 2)) * Fraction(2) ** k < f * Fraction(2) ** -380


def pow_rn(x, y, fmt):
    """Correctly rounded x^y for dyadic x >= 0 and y > 0 (the arguments Listing 5 makes)."""
    if x == 0:
        return 0.0
    if x == 1:
        return 1.0
    fy = F(y)
    b = fy.denominator.bit_length() - 1  # y = a / 2^b
    if b <= 8:
        r = _exact_root(F(x), b)
        if r is not None:
            return rn(r ** fy.numerator, fmt)
    with mpmath.workprec(400):
        v = mpmath.power(mpmath.mpf(x), mpmath.mpf(y))
        assert not _ambiguous(v, fmt), (x, y)  # x^y is irrational here: never that close
        return rn(Fraction(int(v.man)) * Fraction(2) ** int(v.exp), fmt)


def emu_v1_hypot(x, y, fmt):
    X, Y = abs(x), abs(y)
    m, M = fmin(X, Y), fmax(X, Y)
    q = div(m, M, fmt)
    Q = fmax(q, 0.0)
    S = fma_sq1(Q, fmt)
    s = sqrt_rn(S, fmt)
    return mul(M, s, fmt)


def emu_v1_lp(p, x, y, fmt):
    X, Y = abs(x), abs(y)
    m, M = fmin(X, Y), fmax(X, Y)
    q = div(m, M, fmt)
    Q = fmax(q, 0.0)
    half_p = rn(F(p) / 2, fmt)
    inv_p = rn(1 / F(p), fmt)
    S = pow_rn(Q, half_p, fmt)
    Z = fma_sq1(S, fmt)
    C = pow_rn(Z, inv_p, fmt)
    return mul(M, C, fmt)


def _to_fmt(v, fmt):
    """v rounded to fmt (+inf beyond its range)."""
    if fmt == "f64":
        return float(v)
    with np.errstate(over="ignore"):
        return float(np.float32(v))


def pairs(fmt, count, seed):
    """Random pairs over every magnitude ratio and range, plus edge pairs: zeros, equal and
    adjacent operands, ratios at and beyond the precision, subnormal, huge and infinite
    operands."""
    prec, ulp_min, emax = FMTS[fmt]
    rng = random.Random(seed)
    out = []
    big = _to_fmt((2 - 2.0 ** (1 - prec)) * 2.0 ** (emax - 1), fmt)
    tiny = 2.0 ** ulp_min
    edge_vals = [0.0, tiny, 3 * tiny, 2.0 ** (ulp_min + prec - 1), 1.0, 3.0, 4.0, big, big / 2, INF]
    for a in edge_vals:
        for b in edge_vals:
            out.append((a, -b))
    lo, hi = ulp_min + prec, emax - 1
    while len(out) < count:
        ea = rng.randrange(lo - prec - 5, hi + 1)
        a = _to_fmt(math.ldexp(rng.random() + 0.5, ea), fmt)
        kind = rng.random()
        if kind < 0.45:
            b = math.ldexp(rng.random() + 0.5, ea + rng.randrange(-prec - 3, 1))
        elif kind < 0.6:
            b = math.ldexp(rng.random() + 0.5, ea + rng.randrange(-3 * prec, 3))
        elif kind < 0.7:
            b = a * (1 + rng.random() * 2.0 ** -rng.randrange(1, prec))
        elif kind < 0.8:
            b = a
        else:
            b = math.ldexp(rng.random(), rng.randrange(lo - prec, hi + 1))
        b = _to_fmt(b, fmt)
        if math.isinf(a) or math.isinf(b):
            continue
        out.append((a if rng.random() < 0.5 else -a, b if rng.random() < 0.5 else -b))
    return out


def _bits(v, fmt):
    return np.array([v], dtype=np.float32 if fmt == "f32" else np.float64).view(
        np.uint32 if fmt == "f32" else np.uint64)[0]


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_v1_hypot_is_listing2_rounded_per_operation(fmt):
    node = oracle.v1_hypot if fmt == "f64" else oracle.v1_hypotf
    bad = []
    for a, b in pairs(fmt, 100000, 101 if fmt == "f64" else 102):
        want, got = emu_v1_hypot(a, b, fmt), node(a, b)
        if _bits(got, fmt) != _bits(want, fmt):
            bad.append((a, b, got, want))
    assert not bad, (len(bad), bad[:5])


LP_PS = [0.5, 2.0 / 3.0, 1.5, 3.0, 4.5, 8.0]


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", LP_PS)
def test_v1_lp_is_listing5_rounded_per_operation(fmt, p):
    p = _to_fmt(p, fmt)
    node = oracle.v1_lp if fmt == "f64" else oracle.v1_lpf
    bad = []
    for a, b in pairs(fmt, 17000, int(p * 1000) + (7 if fmt == "f32" else 0)):
        want, got = emu_v1_lp(p, a, b, fmt), node(p, a, b)
        if _bits(got, fmt) != _bits(want, fmt):
            bad.append((a, b, got, want))
    assert not bad, (len(bad), bad[:5])
    assert oracle.counters()["pow_unresolved"] == 0


def test_emulation_rounding_primitives():
    """The emulation's own pieces against plain facts: RN agrees with the hardware's
    correctly rounded double and float operations, exact roots are found, and the
    exponent roundings of Sect. 4 are RN(p/2) = p/2 and RN(1/p)."""
    rng = random.Random(5)
    for _ in range(2000):
        a, b = rng.random() * 10, rng.random() * 10 + 1e-3
        assert rn(F(a) / F(b), "f64") == a / b
        fa, fb = np.float32(a), np.float32(b)
        assert rn(F(float(fa)) / F(float(fb)), "f32") == float(fa / fb)
        assert sqrt_rn(a, "f64") == math.sqrt(a)
        assert sqrt_rn(float(fa), "f32") == float(np.sqrt(fa))
    assert rn(F(2) ** 1024, "f64") == INF and rn(F(2) ** 1023, "f64") == 2.0 ** 1023
    assert rn(F(2) ** -1075, "f64") == 0.0 and rn(F(3) * F(2) ** -1076, "f64") == 2.0 ** -1074
    assert rn(F(2) ** -150, "f32") == 0.0 and rn(F(3) * F(2) ** -151, "f32") == 2.0 ** -149
    assert _exact_root(Fraction(81, 256), 2) == Fraction(3, 4) and _exact_root(F(2), 1) is None
    assert pow_rn(15752961 / 2 ** 24, 2.25, "f64") == rn(F(63) ** 9 / F(2) ** 54, "f64")  # an exact tie
    assert rn(1 / F(3.0), "f64") == 1.0 / 3.0 and rn(F(3.0) / 2, "f64") == 1.5
    assert emu_v1_hypot(3.0, 4.0, "f64") == 5.0 and emu_v1_hypot(0.0, 0.0, "f64") == 0.0
    assert emu_v1_hypot(INF, 1.0, "f64") == INF and emu_v1_hypot(INF, INF, "f64") == INF
