"""Pins of the oracle's recursions: tree shapes from the paper's worked examples, bitwise
agreement with the exact-node recursion, closed forms, invariances, Theorem 3 bounds, the
library contract for special inputs, and thread-count independence."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from oracle import bounds, exact

N0 = 1000000  # id of the first internal node in a trace


def test_tree_n7_matches_eq_r():
    # Eq. (r): R([x1..x7]) = h(h(h(x1,x2), h(x3,x4)), h(h(x5,x6), |x7|)), completion order 1..7.
    t = oracle.trace(7)
    assert t == [(1, 2), (3, 4), (N0, N0 + 1), (5, 6), (N0 + 3, 7), (N0 + 2, N0 + 4)]


def test_lane_example_p4_n16():
    # Sect. 3: with 4 lanes and n = 16, lane l holds h(h(x_l, x_l+4), h(x_l+8, x_l+12)).
    t = oracle.trace(16, lanes=4)
    lanes = []
    for lane in range(4):
        a, b, c = t[3 * lane: 3 * lane + 3]
        l1 = lane + 1
        assert a == (l1, l1 + 4) and b == (l1 + 8, l1 + 12)
        assert c == (N0 + 3 * lane, N0 + 3 * lane + 1)
        lanes.append(N0 + 3 * lane + 2)
    # final A over the 4 lane values (Listing 1's tree on 4 elements)
    assert t[12:] == [(lanes[0], lanes[1]), (lanes[2], lanes[3]), (N0 + 12, N0 + 13)]


def test_tail_example_n13_p8():
    # Sect. 3: n = 13, 8 lanes: 2 vectors, the second being the 5-element tail padded with zeros.
    t = oracle.trace(13, lanes=8)
    assert t[:8] == [(1, 9), (2, 10), (3, 11), (4, 12), (5, 13), (6, 0), (7, 0), (8, 0)]


def test_recursion_depth():
    # Sect. 3: recursion depth ceil(lg(max(n/p, 1))) -- for R (p = 1) the tree depth is ceil(lg n).
    for n in [1, 2, 3, 7, 8, 9, 100, 1000, 4097]:
        assert bounds.depth_R(n) == (0 if n == 1 else math.ceil(math.log2(n)))


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_A_is_bitwise_the_exact_node_recursion(fmt):
    dt = np.float64 if fmt == "f64" else np.float32
    for seed, (kind, lo, hi) in enumerate([("u11", 0, 0), ("exp", -20, 20), ("exp", -60, 60),
                                           ("u11exp", -30, 30)]):
        for n in list(range(1, 40)) + [63, 64]:
            x = vnp_gen.np_fill(n, dtype=fmt, kind=kind, lo=lo, hi=hi, seed=seed, stream=n)
            assert oracle.nrmf(x, "A") == dt(exact.R_exact_A(x.tolist(), fmt))
    if fmt == "f64":
        x = vnp_gen.np_fill(50, kind="exp", lo=-1074, hi=-1000, seed=4)
        assert oracle.nrmf(x, "A") == exact.R_exact_A(x.tolist(), fmt)
        x = vnp_gen.np_fill(50, kind="exp", lo=990, hi=1010, seed=4)
        assert oracle.nrmf(x, "A") == exact.R_exact_A(x.tolist(), fmt)


@pytest.mark.parametrize("algo,node", [("A", "cr"), ("H", "v1")])
def test_theorem3_bounds_hold(algo, node):
    for k in [1, 2, 5, 10, 16, 20]:
        n = 1 << k
        x = vnp_gen.host_fill(n, kind="u01", seed=k)
        e = oracle.exact_nrm2(x)
        r = oracle.nrmf(x, algo)
        assert oracle.relerr(r, e, "f64") <= float(bounds.ub_R(n, node)) + 1  # +1: rounding of E itself


def test_observed_error_below_three_eps():
    # Sect. 2 reports relerr < 3 for every recursive algorithm on U(0,1) and N(0,1) inputs.
    x = vnp_gen.host_fill(1 << 20, kind="u01", seed=1)
    e = oracle.exact_nrm2(x)
    for algo in "AHZ":
        assert oracle.relerr(oracle.nrmf(x, algo), e, "f64") < 3
    xs = vnp_gen.host_fill(1 << 20, dtype="f32", kind="u01", seed=1)
    es = oracle.exact_nrm2(xs)
    for algo in "AHZ":
        assert oracle.relerr(oracle.nrmf(xs, algo), es, "f32") < 3


def test_n_copies_closed_form():
    for c in [1.0, 3.0, 0.1, 1e-300, 1e300, 2.0 ** -1070]:
        for n in [2, 3, 4, 16, 100, 1 << 12]:
            x = np.full(n, c)
            want = exact.rn_sqrt_dyadic(*exact._dyadic(n * __import__("fractions").Fraction(c) ** 2))
            r = oracle.nrmf(x, "A")
            if want > 2.0 ** -1000:
                assert oracle.relerr(r, want, "f64") <= float(bounds.ub_R(n, "cr")) + 1
    # 4 copies of 1: h(h(1,1), h(1,1)) = RN(RN(sqrt 2) sqrt 2)
    assert oracle.nrmf(np.ones(4), "A") == oracle.cr_hypot(math.sqrt(2), math.sqrt(2))


def test_range_end_closed_forms():
    big = np.finfo(np.float64).max
    assert oracle.nrmf(np.array([big / 2, big / 2]), "A") < math.inf
    assert oracle.nrmf(np.array([big, big]), "A") == math.inf
    assert oracle.nrmf(np.array([big, 1e-300]), "A") == big
    tiny = 2.0 ** -1074
    assert oracle.nrmf(np.array([3 * tiny, 4 * tiny]), "A") == 5 * tiny


def test_exact_invariances():
    x = vnp_gen.np_fill(1001, kind="exp", lo=-20, hi=20, seed=3)
    r = oracle.nrmf(x, "A")
    assert oracle.nrmf(-x, "A") == r
    s = np.where(np.arange(x.size) % 3 == 0, -x, x)
    assert oracle.nrmf(s, "A") == r
    for k in (-500, -7, 9, 600):
        assert oracle.nrmf(np.ldexp(x, k), "A") == math.ldexp(r, k)
    # sibling swap: the first two leaves are siblings (n = 2 leaf node), so swapping them is exact
    y = x.copy()
    y[[0, 1]] = y[[1, 0]]
    assert oracle.nrmf(y, "A") == r
    # swapping the two halves of a power-of-two-length vector swaps the root's children
    z = vnp_gen.np_fill(1024, kind="exp", lo=-20, hi=20, seed=4)
    assert oracle.nrmf(np.concatenate([z[512:], z[:512]]), "A") == oracle.nrmf(z, "A")


def test_contract_special_inputs():
    assert oracle.nrmf(np.zeros(0), "A") == 0
    assert oracle.nrmf(np.zeros(5), "A") == 0
    assert oracle.nrmf(np.array([1.0, -3.0]), "A") == oracle.cr_hypot(1, 3)
    assert math.isnan(oracle.nrmf(np.array([1.0, np.nan, 2.0]), "A"))
    assert oracle.nrmf(np.array([1.0, -np.inf, 2.0]), "A") == math.inf
    assert math.isnan(oracle.nrmf(np.array([np.inf, np.nan]), "A"))
    assert math.isnan(oracle.nrmp(np.array([np.inf, np.nan]), 3.0))
    assert oracle.nrmp(np.array([np.inf, 1.0]), 3.0) == math.inf
    assert oracle.nrmf(np.array([-2.5]), "A") == 2.5


@pytest.mark.parametrize("algo", ["A", "H", "Z"])
def test_thread_count_does_not_change_bits(algo):
    x = vnp_gen.host_fill(300001, kind="exp", lo=-20, hi=20, seed=8)
    r1 = oracle.nrmf(x, algo, threads=1)
    for t in (2, 3, 8):
        assert oracle.nrmf(x, algo, threads=t) == r1


def test_exact_nrm2_two_routes():
    # superaccumulator + integer sqrt vs Fraction sum, and vs the binary128 route
    for seed in range(5):
        x = vnp_gen.np_fill(200, kind="exp", lo=-300, hi=300, seed=seed)
        assert oracle.exact_nrm2(x) == exact.nrm2_exact(x.tolist())
        with np.errstate(over="ignore"):
            xs = x.astype(np.float32)
        xs = xs[np.isfinite(xs)]
        assert oracle.exact_nrm2(xs) == np.float32(exact.nrm2_exact(xs.tolist(), "f32"))
    x = vnp_gen.host_fill(1 << 18, kind="exp", lo=-20, hi=20, seed=1)
    hi, lo = oracle.ref_pnorm(x, 2.0)
    assert oracle.exact_nrm2(x) == hi


def test_Z_with_one_lane_is_H():
    x = vnp_gen.np_fill(777, kind="exp", lo=-10, hi=10, seed=2)
    assert oracle.nrmf(x, "Z", lanes=1) == oracle.nrmf(x, "H")


def test_pnorm_reductions():
    x = vnp_gen.np_fill(501, kind="exp", lo=-10, hi=10, seed=6)
    # p = 2 through Listing 5 is the H recursion (Eq. (sp))
    assert oracle.nrmp(x, 2.0) == oracle.nrmf(x, "H")
    # p = 1 on small integers is the exact sum
    ints = np.arange(-50, 51, dtype=np.float64)
    assert oracle.nrmp(ints, 1.0) == np.abs(ints).sum()
    assert oracle.nrmp(x, math.inf) == np.abs(x).max()
    # integer-p results within the empirical tolerance of the binary128 reference
    for p in (1.5, 3.0, 4.5, 8.0):
        r = oracle.nrmp(x, p)
        hi, lo = oracle.ref_pnorm(x, p)
        assert oracle.relerr(r, hi, "f64") < bounds.tol_parity(x.size) / 2.0 ** -53
    assert oracle.counters()["pow_unresolved"] == 0
