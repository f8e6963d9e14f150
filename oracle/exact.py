"""Exact references in Python big integers -- TEST INFRASTRUCTURE ONLY.

These are the "obviously correct" definitions the C oracle is pinned against:

* ``rn_sqrt_dyadic(N, E, fmt)``: RN(sqrt(N * 2**E)) in binary64 or binary32, with
  subnormal results, overflow to +inf and ties to even -- the rounding of the exact
  Frobenius norm (Sect. 2, the "exact" norm of the tester, computed here exactly
  instead of with 2048-bit MPFR).
* ``cr_hypot_exact(x, y, fmt)``: the correctly rounded hypotenuse (Eq. (hypot) with
  |eps_h| <= eps, Table 2's cr_hypot), from the exact rational x^2 + y^2.
* ``nrm2_exact(xs, fmt)``: RN(sqrt(sum x_i^2)) for a list of floats.
* ``R_exact_A(xs, fmt)``: the scalar recursion R of Sect. 2 (ceil split; n = 1 gives
  |x|, n = 2 one node) with every node ``cr_hypot_exact`` -- the A algorithm, unique
  because every node is correctly rounded.
"""
from __future__ import annotations

import math
from fractions import Fraction

FMT = {
    # precision p (bits), minimum exponent of the ulp (subnormal grid), emax
    "f64": (53, -1074, 1024),
    "f32": (24, -149, 128),
}


def _to_float(mant: int, exp: int, fmt: str) -> float:
    if fmt == "f64":
        return math.ldexp(mant, exp)
    import numpy as np

    return float(np.float32(math.ldexp(mant, exp)))


def rn_sqrt_dyadic(N: int, E: int, fmt: str = "f64") -> float:
    """Correctly rounded sqrt(N * 2**E) for an integer N >= 0, in format ``fmt``."""
    prec, ulp_min, emax = FMT[fmt]
    if N < 0:
        raise ValueError("negative")
    if N == 0:
        return 0.0
    if E % 2:
        N <<= 1
        E -= 1
    # sqrt(N 2^E) = sqrt(N) 2^(E/2), and floor(log2(sqrt(N))) = floor((bitlen(N) - 1) / 2).
    lg = (N.bit_length() - 1) // 2 + E // 2
    k = max(lg - (prec - 1), ulp_min)  # exponent of the result's ulp
    # q = floor(sqrt(S) / 2^(k-2)): the result's bits plus two guard bits.
    sh = E - 2 * (k - 2)  # S / 4^(k-2) = N 2^sh
    if sh >= 0:
        T, lost = N << sh, False
    else:
        T, lost = N >> (-sh), (N & ((1 << (-sh)) - 1)) != 0
    q = math.isqrt(T)
    exact = (q * q == T) and not lost
    mant, rem = q >> 2, q & 3
    if rem > 2 or (rem == 2 and not exact) or (rem == 2 and exact and (mant & 1)):
        mant += 1
    if mant.bit_length() > prec:  # rounding carried into a new binade
        mant >>= 1
        k += 1
    if mant.bit_length() + k > emax:
        return math.inf
    return _to_float(mant, k, fmt)


def _dyadic(fr: Fraction):
    """Fraction with a power-of-two denominator -> (N, E) with fr = N 2^E."""
    d = fr.denominator
    assert d & (d - 1) == 0
    return fr.numerator, -(d.bit_length() - 1)


def cr_hypot_exact(x: float, y: float, fmt: str = "f64") -> float:
    if math.isinf(x) or math.isinf(y):
        return math.inf
    if math.isnan(x) or math.isnan(y):
        return math.nan
    s = Fraction(x) ** 2 + Fraction(y) ** 2
    N, E = _dyadic(s)
    return rn_sqrt_dyadic(N, E, fmt)


def nrm2_exact(xs, fmt: str = "f64") -> float:
    s = sum((Fraction(float(v)) ** 2 for v in xs), Fraction(0))
    if s == 0:
        return 0.0
    N, E = _dyadic(s)
    return rn_sqrt_dyadic(N, E, fmt)


def R_exact_A(xs, fmt: str = "f64") -> float:
    """The A recursion with exactly rounded nodes (Listing 1's split)."""
    xs = [float(v) for v in xs]

    def rec(lo, n):
        if n == 1:
            return abs(xs[lo])
        if n == 2:
            return cr_hypot_exact(xs[lo], xs[lo + 1], fmt)
        p = (n >> 1) + (n & 1)
        return cr_hypot_exact(rec(lo, p), rec(lo + p, n - p), fmt)

    return rec(0, len(xs))


def limbs_to_int(limbs) -> int:
    v = 0
    for i, w in enumerate(limbs):
        v |= int(w) << (64 * i)
    return v
