"""Oracle for the norm of a multi-dimensional array with a leading dimension (Sect. 3.1):
pinned by exact rational arithmetic on tiny arrays, by closed forms, by the contiguous-
array identity of Sect. 3.1 and by never reading the rows past m."""
import math

import numpy as np
import pytest

import oracle
from oracle import bounds, exact


def colmajor(cols, lda, fill=np.nan, dtype=np.float64):
    """Column-major storage of the given columns with leading dimension lda (padding rows
    hold `fill`)."""
    m = len(cols[0])
    a = np.full(lda * len(cols), fill, dtype=dtype)
    for j, c in enumerate(cols):
        a[j * lda:j * lda + m] = c
    return a


@pytest.mark.parametrize("m,ncols", [(1, 2), (2, 3), (3, 5), (5, 4), (7, 7)])
def test_exact_composition_on_tiny_arrays(m, ncols):
    """Column norms by the exactly rounded recursion, then the same over the column norms:
    bitwise equal (exact rationals, independent of the oracle's binary128 node)."""
    rng = np.random.default_rng(100 * m + ncols)
    for _ in range(20):
        cols = [np.ldexp(rng.uniform(-1, 1, m), rng.integers(-40, 40, m)) for _ in range(ncols)]
        a = colmajor(cols, m + 3)
        want = exact.R_exact_A([exact.R_exact_A(c) for c in cols])
        assert oracle.nrm_mat(a, m, ncols, m + 3) == want


def test_padding_rows_are_never_read():
    cols = [np.array([3.0, 0.0]), np.array([4.0, 0.0])]
    for fill in (np.nan, np.inf, 1e300):
        assert oracle.nrm_mat(colmajor(cols, 5, fill), 2, 2, 5) == 5.0


def test_pythagorean_column_norms():
    # column norms 3, 4 -> 5; norms 3, 4, 12, 0 -> node(node(3, 4), node(12, 0)) = 13
    for k in (-1000, -3, 0, 7, 900):
        s = 2.0 ** k
        cols = [np.array([3.0 * s, 0.0, 0.0]), np.array([0.0, -4.0 * s, 0.0])]
        assert oracle.nrm_mat(colmajor(cols, 4), 3, 2, 4) == 5.0 * s
        cols = [np.array([0.0, 3.0 * s]), np.array([4.0 * s, 0.0]), np.array([0.0, -12.0 * s]), np.zeros(2)]
        assert oracle.nrm_mat(colmajor(cols, 3), 2, 4, 3) == 13.0 * s


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_contiguous_array_is_one_vector(dtype):
    rng = np.random.default_rng(7)
    a = rng.uniform(-1, 1, 60 * 70).astype(dtype)
    assert oracle.nrm_mat(a, 60, 70, 60) == oracle.nrmf(a)
    assert oracle.nrm_mat(a, 60, 70, 60, p=3.0) == oracle.nrmp(a, 3.0)


@pytest.mark.parametrize("m,ncols", [(1000, 37), (3, 4097), (8193, 5)])
def test_constant_array_closed_form_and_exact_bound(m, ncols):
    c = 0.7853981633974483
    a = colmajor([np.full(m, c)] * ncols, m + 11)
    got = float(oracle.nrm_mat(a, m, ncols, m + 11))
    ex = float(oracle.exact_nrm2(np.full(m * ncols, c)))
    assert ex == float(np.float64(c * math.sqrt(m * ncols))) or abs(ex - c * math.sqrt(m * ncols)) <= 2 ** -52 * ex
    depth = bounds.depth_R(m) + bounds.depth_R(ncols)
    assert abs(got - ex) <= depth * 2.0 ** -53 * ex * (1 + 1e-12)


def test_single_nonzero_column_is_that_columns_norm():
    rng = np.random.default_rng(3)
    col = np.ldexp(rng.uniform(-1, 1, 777), rng.integers(-5, 5, 777))
    cols = [np.zeros(777)] * 6
    cols[4] = col
    assert oracle.nrm_mat(colmajor(cols, 800), 777, 6, 800) == oracle.nrmf(col)


def test_pnorm_reductions():
    rng = np.random.default_rng(5)
    cols = [rng.integers(-9, 9, 11).astype(np.float64) for _ in range(13)]
    a = colmajor(cols, 12)
    assert oracle.nrm_mat(a, 11, 13, 12, p=1.0) == float(sum(np.abs(c).sum() for c in cols))
    assert oracle.nrm_mat(a, 11, 13, 12, p=math.inf) == max(np.abs(c).max() for c in cols)


def test_empty_and_invalid():
    assert oracle.nrm_mat(np.zeros(4), 0, 3, 1) == 0.0
    assert oracle.nrm_mat(np.zeros(4), 2, 0, 2) == 0.0
    with pytest.raises(ValueError):
        oracle.nrm_mat(np.zeros(8), 4, 2, 3)
