"""Constants of the p-node evaluation in vnp_nodes_p.hpp.

Chebyshev interpolation in 60-digit arithmetic (a near-minimax fit), then rounding to
binary64; prints each polynomial coefficient as a C hex-float literal with the largest
error of the rounded polynomial, evaluated by Horner's rule in exact arithmetic on a dense
grid, and writes the tables to vnp_lp_table.hpp: the log2 table and the reduction table of
the power Z^(1/p) (whose p-dependent values the library computes per p).

    python paper_2509_06220_amd/csrc/lp_coeffs.py
"""
import os

import mpmath as mp

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))
TAB_BITS = 7            # fraction bits of v in [1/2, 1) that pick the table entry
T_MAX = mp.mpf(2) ** -8 * mp.mpf("1.01")  # |t| bound of the reduced argument, with margin


def cheb_fit(f, a, b, deg):
    """Power-basis coefficients c[0..deg] of the degree-deg Chebyshev interpolant of f on [a, b]."""
    nodes = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (deg + 1)) for k in range(deg + 1)]
    vals = [f(x) for x in nodes]
    A = mp.matrix([[x ** j for j in range(deg + 1)] for x in nodes])
    return list(mp.lu_solve(A, mp.matrix(vals)))


def horner(cs, x):
    r = mp.mpf(0)
    for c in reversed(cs):
        r = r * x + mp.mpf(c)
    return r


def worst(err, a, b, npts=4000):
    return max(err(a + (b - a) * i / npts) for i in range(npts + 1))


def table():
    """Entry j: c_j = RN(1 / mid_j), mid_j = 1/2 + (j + 1/2) / 2^(TAB_BITS+1), the centre of the
    j-th interval of [1/2, 1); l_j = RN(log2(2 / c_j)) in [0, 1)."""
    rows = []
    for j in range(1 << TAB_BITS):
        mid = mp.mpf(1) / 2 + (mp.mpf(j) + mp.mpf(1) / 2) / 2 ** (TAB_BITS + 1)
        c = float(1 / mid)
        rows.append((c, float(mp.log(2 / mp.mpf(c), 2))))
        # every v of the interval has |v c_j - 1| <= T_MAX
        lo, hi = mp.mpf(1) / 2 + mp.mpf(j) / 2 ** (TAB_BITS + 1), mp.mpf(1) / 2 + mp.mpf(j + 1) / 2 ** (TAB_BITS + 1)
        assert max(abs(lo * mp.mpf(c) - 1), abs(hi * mp.mpf(c) - 1)) <= T_MAX
    return rows


def main():
    # 2^f, |f| <= 1/2, degree 11 (exact at 0)
    e = [float(c) for c in cheb_fit(lambda f: mp.mpf(2) ** f, mp.mpf(-0.5), mp.mpf(0.5), 11)]
    e[0] = 1.0
    w = worst(lambda f: abs(horner(e, f) / mp.mpf(2) ** f - 1), mp.mpf(-0.5), mp.mpf(0.5))
    print(f"// 2^f, |f| <= 1/2, degree 11: max relative error {mp.nstr(w, 3)} (2^{mp.nstr(mp.log(w, 2), 4)})")
    for j, c in enumerate(e):
        print(f"    {c.hex()},  // f^{j}")
    # log2(1 + t) = t g(t), |t| <= T_MAX, g of degree 5
    g = [float(c) for c in cheb_fit(lambda t: mp.log(1 + t, 2) / t if t != 0 else 1 / mp.log(2), -T_MAX, T_MAX, 5)]
    w = worst(lambda t: abs(t * horner(g, t) - mp.log(1 + t, 2)), -T_MAX, T_MAX)
    print(f"// log2(1 + t) = t g(t), |t| <= 1.01 * 2^-8: max absolute error {mp.nstr(w, 3)} "
          f"(2^{mp.nstr(mp.log(w, 2), 4)})")
    for j, c in enumerate(g):
        print(f"    {c.hex()},  // t^{j}")
    # (1 + t)^a = 1 + t (b_1 + b_2 t + ... + b_7 t^6), |t| < 2^-7, a <= 2: the series is
    # evaluated with the binomial coefficients of a, computed per p by the library; the
    # first omitted term is |b_8| t^8 < 2^-56 |b_8| with |b_8| <= 1/8 for a in (0, 2]
    bmax = max(abs(mp.binomial(mp.mpf(a) / 64, 8)) for a in range(1, 129))
    print(f"// (1 + t)^a, |t| < 2^-7, a in (0, 2]: first omitted term <= 2^{mp.nstr(mp.log(bmax * mp.mpf(2) ** -56, 2), 4)}")
    rows = table()
    worst_l = max(abs(mp.mpf(l) - mp.log(2 / mp.mpf(c), 2)) for c, l in rows)
    print(f"// table: {len(rows)} entries, max |l_j - log2(2 / c_j)| = 2^{mp.nstr(mp.log(worst_l, 2), 4)}")
    path = os.path.join(HERE, "vnp_lp_table.hpp")
    with open(path, "w") as fh:
        fh.write("// Table of the binary64 log2 in vnp_nodes_p.hpp, written by lp_coeffs.py (do not edit).\n")
        fh.write(f"// Entry j (the top {TAB_BITS} fraction bits of v in [1/2, 1)): {{c_j, l_j}} with\n")
        fh.write(f"// c_j = RN(1 / mid_j), mid_j = 1/2 + (j + 1/2) / {2 ** (TAB_BITS + 1)}, and "
                 "l_j = RN(log2(2 / c_j)).\n")
        fh.write(f"// Power table (Z^(1/p) for Z in [1, 2)): entry j (the top {TAB_BITS} fraction bits of Z)\n")
        fh.write(f"// is c'_j = RN({2 ** TAB_BITS} / ({2 ** TAB_BITS} + j)), the reciprocal of the interval's left end.\n")
        fh.write("#pragma once\n\nnamespace vnp {\n\n")
        fh.write(f"constexpr int LP_TAB_BITS = {TAB_BITS};\n")
        fh.write("#define VNP_LP_LOG_TAB \\\n    { \\\n")
        for c, l in rows:
            fh.write(f"        {{{c.hex()}, {l.hex()}}}, \\\n")
        fh.write("    }\n")
        fh.write("#define VNP_LP_POW_TAB \\\n    { \\\n")
        for j in range(1 << TAB_BITS):
            fh.write(f"        {float(mp.mpf(2 ** TAB_BITS) / (2 ** TAB_BITS + j)).hex()}, \\\n")
        fh.write("    }\n")
        fh.write("static __constant__ double lp_tab_src[1 << LP_TAB_BITS][2] = VNP_LP_LOG_TAB;\n")
        fh.write("static __constant__ double lp_ptab_src[1 << LP_TAB_BITS] = VNP_LP_POW_TAB;\n")
        fh.write("static const double lp_ptab_host[1 << LP_TAB_BITS] = VNP_LP_POW_TAB;\n")
        fh.write("\n}  // namespace vnp\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
