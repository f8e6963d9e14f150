"""The bound calculator reproduces every printed digit of Table 3 (Sect. 2)."""
import os

import mpmath
import pytest

from oracle import bounds

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3.txt")


def _rows():
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, L, A, H = line.split()
                yield int(k), L, A, H


def _same_18_digits(value, printed):
    return mpmath.nstr(value, 18, min_fixed=1, max_fixed=0) == mpmath.nstr(mpmath.mpf(printed), 18, min_fixed=1,
                                                                           max_fixed=0)


@pytest.mark.parametrize("k,L,A,H", list(_rows()))
def test_table3_row(k, L, A, H):
    n = 1 << k
    assert _same_18_digits(bounds.ub_L(n), L)
    assert _same_18_digits(bounds.ub_R(n, "cr"), A)
    assert _same_18_digits(bounds.ub_R(n, "v1"), H)


def test_literal_eq8_disagrees_with_table3():
    # Documented reading: Eq. (8) as printed gives about 4 at n = 4, Table 3 prints 2.00000000000000011.
    assert 3.9 < float(bounds.ub_R_literal(4, "cr")) < 4.1
    assert abs(float(bounds.ub_R(4, "cr")) - 2.0) < 1e-15


def test_tolerance_formula():
    assert bounds.tol_parity(1) == 2 * 2.0 ** -53
    assert bounds.tol_parity(1 << 30) == 62 * 2.0 ** -53
    assert bounds.tol_parity(1 << 30, "f32") == 62 * 2.0 ** -24
