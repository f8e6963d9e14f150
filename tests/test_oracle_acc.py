"""Oracle for Theorem 1's single-accumulator algorithm (the baseline of the accuracy study):
pinned by an exact emulation of each fma, Pythagorean sums, Theorem 1's bound, and error
growth beyond the recursion's."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle


def acc_exact(xs):
    """fma(x, x, g) rounded once per step (Fraction arithmetic, correctly rounded by float())."""
    g = 0.0
    for v in xs:
        g = float(Fraction(float(v)) ** 2 + Fraction(g))
    return math.sqrt(g)


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_exact_emulation(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        x = np.ldexp(rng.uniform(-1, 1, n), rng.integers(-30, 30, n))
        assert oracle.nrm_acc(x) == acc_exact(x)


def test_pythagorean_sums():
    assert oracle.nrm_acc(np.array([3.0, 4.0])) == 5.0
    assert oracle.nrm_acc(np.array([1.0, 2.0, 2.0])) == 3.0
    assert oracle.nrm_acc(np.array([2.0, 3.0, 6.0], dtype=np.float32)) == np.float32(7.0)


@pytest.mark.parametrize("fmt,n", [("f64", 1 << 20), ("f32", 1 << 16)])
def test_theorem1_bound_and_linear_growth(fmt, n):
    dt = np.float64 if fmt == "f64" else np.float32
    eps = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    x = np.full(n, 0.1, dtype=dt)
    ex = float(oracle.exact_nrm2(x))
    acc = float(oracle.nrm_acc(x))
    bound = math.expm1((n / 2 + 1) * math.log1p(eps))  # sqrt((1 + eps)^n) (1 + eps) - 1, Eq. (13)
    assert abs(acc - ex) / ex <= bound * (1 + 1e-9)
    # the single accumulator loses far more than the recursion on the same data
    tree = float(oracle.nrmf(x, "A"))
    assert abs(acc - ex) / ex > 50 * eps and abs(tree - ex) / ex < 4 * eps
