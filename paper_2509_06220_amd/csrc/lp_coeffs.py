"""Constants of the p-node evaluation in vnp_nodes_p.hpp.

Chebyshev interpolation in 60-digit arithmetic (a near-minimax fit), then rounding to
binary64; prints each polynomial's largest error, evaluated by Horner's rule in exact
arithmetic on a dense grid, and writes the tables and coefficients to vnp_lp_table.hpp:

* log2 f for f in [1/2, 1]: 2^LOG_BITS intervals and f = 1, entry {c_j, l_j} with c_j = RN(1/mid_j)
  and l_j = RN(log2(2/c_j)), except entry 0, which takes the interval's left end:
  c_0 = 2, l_0 = 0, so that f = 1/2 gives t = 0 and log2(2 f) = 0 exactly; then
  log2 f = (l_j - 1) + log2(1 + t), t = f c_j - 1, and log2(1 + t) = t g(t), with g fitted
  on [-T_MAX, 2 T_MAX] (entry 0's t lies in [0, 2^-LOG_BITS));
* 2^y in steps of 1/2^EXP_BITS: entry j is T_j = RN(2^(j / 2^EXP_BITS));
  2^(u / 2^EXP_BITS) - 1 = u H(u) for |u| <= 1/2 (H's
  coefficients are those of (2^r - 1) / r in r = u / 2^EXP_BITS, scaled exactly by powers
  of two);
* Z^a for Z in [1, 2): 2^POW_BITS intervals, c'_j = RN(2^POW_BITS / (2^POW_BITS + j)),
  the reciprocal of the interval's left end (the p-dependent values R_j = (1/c'_j)^a' are
  computed by the library per p).

    python paper_2509_06220_amd/csrc/lp_coeffs.py
"""
import os

import mpmath as mp

mp.mp.dps = 60
HERE = os.path.dirname(os.path.abspath(__file__))
LOG_BITS = 10  # fraction bits of f in [1/2, 1) that pick the log2 table entry
LOG_DEG = 3    # degree of g
EXP_BITS = 9   # 2^y table: 2^EXP_BITS entries per octave
EXP_DEG = 3    # degree of H
POW_BITS = 9   # fraction bits of Z in [1, 2) that pick the power table entry
POW_TERMS = 5  # binomial terms b_1 .. b_POW_TERMS of (1 + t)^a'
T_MAX = mp.mpf(2) ** -(LOG_BITS + 1) * mp.mpf("1.01")  # |t| bound of the reduced log argument, with margin


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


def log_table():
    rows = []
    for j in range(1 << LOG_BITS):
        lo, hi = mp.mpf(1) / 2 + mp.mpf(j) / 2 ** (LOG_BITS + 1), mp.mpf(1) / 2 + mp.mpf(j + 1) / 2 ** (LOG_BITS + 1)
        if j == 0:  # left end: f = 1/2 maps to t = 0 and log2(2 f) = 0 exactly
            rows.append((2.0, 0.0))
            assert 0 <= hi * 2 - 1 <= 2 * T_MAX
            continue
        mid = mp.mpf(1) / 2 + (mp.mpf(j) + mp.mpf(1) / 2) / 2 ** (LOG_BITS + 1)
        c = float(1 / mid)
        rows.append((c, float(mp.log(2 / mp.mpf(c), 2))))
        # every f of the interval has |f c_j - 1| <= T_MAX
        assert max(abs(lo * mp.mpf(c) - 1), abs(hi * mp.mpf(c) - 1)) <= T_MAX
    rows.append((1.0, 1.0))  # f = 1 (index 2^LOG_BITS, with the exponent's low bit): log2(2 f) = 1
    return rows


def exp_table():
    return [float(mp.mpf(2) ** (mp.mpf(j) / 2 ** EXP_BITS)) for j in range(1 << EXP_BITS)]


def pow_table():
    return [float(mp.mpf(2 ** POW_BITS) / (2 ** POW_BITS + j)) for j in range(1 << POW_BITS)]


def carr(name, vals):
    lines = [", ".join(v.hex() for v in vals[i:i + 4]) for i in range(0, len(vals), 4)]
    body = ",\n    ".join(lines)
    return f"static __constant__ double {name}[{len(vals)}] = {{\n    {body}}};\n"


def main():
    # log2(1 + t) = t g(t), |t| <= T_MAX
    # (log1p and expm1: a Chebyshev node at or near 0 must not cancel)
    g = [float(c) for c in cheb_fit(lambda t: mp.log1p(t) / t / mp.log(2) if t != 0 else 1 / mp.log(2), -T_MAX,
                                    2 * T_MAX, LOG_DEG)]
    wg = worst(lambda t: abs(t * horner(g, t) - mp.log(1 + t, 2)), -T_MAX, 2 * T_MAX)
    print(f"log2(1 + t) = t g(t), -1.01 * 2^-{LOG_BITS + 1} <= t <= 1.01 * 2^-{LOG_BITS}, degree {LOG_DEG}: "
          f"max absolute error 2^{mp.nstr(mp.log(wg, 2), 4)}")
    # (2^r - 1) / r on |r| <= 2^-(EXP_BITS + 1), then scaled to u = r 2^EXP_BITS
    R = mp.mpf(2) ** -(EXP_BITS + 1)
    h = [float(c) for c in cheb_fit(lambda r: mp.expm1(r * mp.log(2)) / r if r != 0 else mp.log(2), -R, R, EXP_DEG)]
    wh = worst(lambda r: abs((1 + r * horner(h, r)) / mp.mpf(2) ** r - 1), -R, R)
    print(f"2^r = 1 + r h(r), |r| <= 2^-{EXP_BITS + 1}, degree {EXP_DEG}: max relative error "
          f"2^{mp.nstr(mp.log(wh, 2), 4)}")
    H = [c * 2.0 ** (-EXP_BITS * (i + 1)) for i, c in enumerate(h)]  # exact power-of-two scaling
    # (1 + t)^a, |t| < 2^-POW_BITS, a in (0, 2]: first omitted binomial term
    bmax = max(abs(mp.binomial(mp.mpf(a) / 64, POW_TERMS + 1)) for a in range(1, 129))
    tb = mp.log(bmax * mp.mpf(2) ** (-POW_BITS * (POW_TERMS + 1)), 2)
    print(f"(1 + t)^a, |t| < 2^-{POW_BITS}, a in (0, 2], {POW_TERMS} terms: first omitted term <= "
          f"2^{mp.nstr(tb, 4)}")
    lrows, erows, prows = log_table(), exp_table(), pow_table()
    wl = max(abs(mp.mpf(l) - mp.log(2 / mp.mpf(c), 2)) for c, l in lrows)
    print(f"log2 table: {len(lrows)} entries, max |l_j - log2(2 / c_j)| = 2^{mp.nstr(mp.log(wl, 2), 4)}")
    path = os.path.join(HERE, "vnp_lp_table.hpp")
    with open(path, "w") as fh:
        fh.write("// Tables and coefficients of the binary64 p node in vnp_nodes_p.hpp, written by lp_coeffs.py\n")
        fh.write("// (do not edit).\n")
        fh.write(f"// log2: entry j (the top {LOG_BITS} fraction bits of f in [1/2, 1)) is {{c_j, l_j}}, c_j =\n")
        fh.write(f"// RN(1 / mid_j), mid_j = 1/2 + (j + 1/2) / {2 ** (LOG_BITS + 1)}, l_j = RN(log2(2 / c_j)), "
                 f"except c_0 = 2, l_0 = 0\n// (the left end: log2(2 f) = 0 exactly at f = 1/2); "
                 f"log2(1 + t) = t g(t), -1.01 * 2^-{LOG_BITS + 1} <= t <=\n// 1.01 * 2^-{LOG_BITS}, "
                 f"g of degree {LOG_DEG} (absolute error 2^{mp.nstr(mp.log(wg, 2), 3)}).  Entry {2 ** LOG_BITS} "
                 f"(f = 1, picked\n// through the exponent's low bit) is {{1, 1}}: log2(2 f) = 1 exactly.\n")
        fh.write(f"// 2^y: entry j is T_j = RN(2^(j / {2 ** EXP_BITS})); 2^(u / {2 ** EXP_BITS}) - 1 = u H(u), "
                 f"|u| <= 1/2, H of degree\n// {EXP_DEG} (relative error 2^{mp.nstr(mp.log(wh, 2), 3)}).\n")
        fh.write(f"// Z^a: entry j (the top {POW_BITS} fraction bits of Z in [1, 2)) is c'_j = "
                 f"RN({2 ** POW_BITS} / ({2 ** POW_BITS} + j)),\n// the reciprocal of the interval's left end; "
                 f"binomial series of {POW_TERMS} terms (first omitted term\n// <= 2^{mp.nstr(tb, 3)}).\n")
        fh.write("#pragma once\n\nnamespace vnp {\n\n")
        fh.write(f"constexpr int LP_LOG_BITS = {LOG_BITS};\nconstexpr int LP_EXP_BITS = {EXP_BITS};\n"
                 f"constexpr int LP_EXP_DEG = {EXP_DEG};\n"
                 f"constexpr int LP_POW_BITS = {POW_BITS};\nconstexpr int LP_POW_TERMS = {POW_TERMS};\n")
        fh.write("static __constant__ double lp_log_src[(1 << LP_LOG_BITS) + 1][2] = {\n")
        for c, l in lrows:
            fh.write(f"    {{{c.hex()}, {l.hex()}}},\n")
        fh.write("};\n")
        fh.write(carr("lp_exp_src", erows))
        fh.write("#define VNP_LP_POW_TAB \\\n    { \\\n")
        for v in prows:
            fh.write(f"        {v.hex()}, \\\n")
        fh.write("    }\n")
        fh.write("static __constant__ double lp_pow_src[1 << LP_POW_BITS] = VNP_LP_POW_TAB;\n")
        fh.write("static const double lp_pow_host[1 << LP_POW_BITS] = VNP_LP_POW_TAB;\n")
        fh.write("// g: coefficients of t^" + str(LOG_DEG) + " .. t^0\n")
        fh.write(carr("lp_log_g", list(reversed(g))))
        fh.write("// H: coefficients of u^" + str(EXP_DEG) + " .. u^0\n")
        fh.write(carr("lp_exp_h", list(reversed(H))))
        fh.write("\n}  // namespace vnp\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
