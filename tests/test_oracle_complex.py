"""Oracle for the norm of a complex vector (the real view of re and im parts, Sect. 1):
pinned by exact rational arithmetic, closed forms, the library norm as a special case, and
the stride conventions."""
import math

import numpy as np
import pytest

import oracle
from oracle import bounds, exact


def test_single_elements_are_exact():
    for k in (-1070, -20, 0, 33, 1000):
        s = 2.0 ** k
        assert oracle.nrmf_complex(np.array([3 * s + 4j * s])) == 5 * s
        assert oracle.nrmf_complex(np.array([-5 * s - 12j * s, 0j])) == 13 * s
    assert oracle.nrmf_complex(np.array([3 + 4j], dtype=np.complex64)) == np.float32(5.0)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13])
def test_exact_rational_recursion_over_the_real_view(n):
    rng = np.random.default_rng(n)
    for _ in range(10):
        re = np.ldexp(rng.uniform(-1, 1, n), rng.integers(-30, 30, n))
        im = np.ldexp(rng.uniform(-1, 1, n), rng.integers(-30, 30, n))
        view = np.empty(2 * n)
        view[0::2], view[1::2] = re, im
        assert oracle.nrmf_complex(re + 1j * im) == exact.R_exact_A(view)


@pytest.mark.parametrize("n", [1000, 4097])
def test_constant_vector_and_library_norm(n):
    c = 0.3
    z = np.full(n, c + 1j * c)
    got = float(oracle.nrmf_complex(z))
    tol = bounds.tol_parity(2 * n, "f64")
    assert abs(got - c * math.sqrt(2 * n)) <= tol * got
    rng = np.random.default_rng(n)
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert abs(float(oracle.nrmf_complex(w)) - np.linalg.norm(w)) <= tol * np.linalg.norm(w)


def test_strides_select_logical_elements():
    rng = np.random.default_rng(9)
    z = rng.standard_normal(301) + 1j * rng.standard_normal(301)
    assert oracle.nrmf_complex(z, incz=3) == oracle.nrmf_complex(z[::3].copy())
    assert oracle.nrmf_complex(z, incz=-2, n=151) == oracle.nrmf_complex(z[::2][::-1].copy())
    assert oracle.nrmf_complex(np.zeros(0, dtype=complex)) == 0.0
