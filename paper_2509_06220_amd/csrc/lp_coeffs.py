"""Coefficients of the polynomial approximations in vnp_nodes_p.hpp.

Chebyshev interpolation in 60-digit arithmetic (a near-minimax fit), then rounding to
binary64; prints each coefficient as a C hex-float literal and the largest relative error
of the rounded polynomial, evaluated by Horner's rule in exact arithmetic, on a dense grid.

    python paper_2509_06220_amd/csrc/lp_coeffs.py
"""
import mpmath as mp

mp.mp.dps = 60


def cheb_fit(f, a, b, deg):
    """Power-basis coefficients c[0..deg] of the degree-deg Chebyshev interpolant of f on [a, b]."""
    nodes = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (deg + 1)) for k in range(deg + 1)]
    vals = [f(x) for x in nodes]
    # solve the Vandermonde system in high precision (small degree, well enough conditioned here)
    A = mp.matrix([[x ** j for j in range(deg + 1)] for x in nodes])
    return list(mp.lu_solve(A, mp.matrix(vals)))


def to_double(c):
    return float(c)


def horner(cs, x):
    r = mp.mpf(0)
    for c in reversed(cs):
        r = r * x + mp.mpf(c)
    return r


def report(name, cs, f, a, b):
    worst = mp.mpf(0)
    for i in range(4001):
        x = a + (b - a) * i / 4000
        fx = f(x)
        if fx != 0:
            worst = max(worst, abs(horner(cs, x) - fx) / abs(fx))
    print(f"// {name}: max relative error of the rounded polynomial {mp.nstr(worst, 3)} "
          f"({mp.nstr(worst / mp.mpf(2) ** -53, 3)} ulp of 2^-53)")
    for j, c in enumerate(cs):
        print(f"    {c.hex()},  // x^{j}")


# exp(x) on |x| <= ln(2) / 2, degree 11
LN2 = mp.log(2)
e = [to_double(c) for c in cheb_fit(mp.exp, -LN2 / 2, LN2 / 2, 11)]
e[0] = 1.0  # exact at 0
report("exp(x), |x| <= ln2/2, degree 11", e, mp.exp, -LN2 / 2, LN2 / 2)

# log2(r) = s * g(s^2), s = (r - 1) / (r + 1), r in [sqrt(1/2), sqrt(2)]: g(u) = 2 atanh(sqrt u) / (sqrt u ln 2)
SMAX = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)


def g(u):
    if u == 0:
        return 2 / LN2
    return 2 * mp.atanh(mp.sqrt(u)) / (mp.sqrt(u) * LN2)


gc = [to_double(c) for c in cheb_fit(g, mp.mpf(0), SMAX ** 2, 7)]
report("2 atanh(s) / (s ln 2) as a polynomial in u = s^2, u <= 0.0295, degree 7", gc, g, mp.mpf(0), SMAX ** 2)
