"""Oracle for the Schatten p-norm (Sect. 4: the p-norm of the singular values), pinned by
unitary invariance (p = 2 is the Frobenius norm of the entries), rank-one and diagonal
matrices, a 2 x 2 closed form of the nuclear norm, and orthogonal invariance."""
import math

import numpy as np
import pytest

import oracle

EPS = 2.0 ** -53


def colmajor(G, lda):
    m, n = G.shape
    a = np.full(lda * n, np.nan)
    for j in range(n):
        a[j * lda:j * lda + m] = G[:, j]
    return a


@pytest.mark.parametrize("m,n", [(8, 8), (37, 20), (20, 37), (64, 64)])
def test_p2_is_the_frobenius_norm(m, n):
    G = np.random.default_rng(m * n).standard_normal((m, n))
    got = float(oracle.schatten(colmajor(G, m + 3), m, n, m + 3, 2.0))
    assert abs(got - float(oracle.exact_nrm2(G.ravel()))) <= 50 * max(m, n) * EPS * got


def test_rank_one_and_diagonal():
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(30), rng.standard_normal(17)
    G = np.outer(u, v)
    s1 = float(np.linalg.norm(u) * np.linalg.norm(v))
    for p in (1.0, 3.0, math.inf):
        got = float(oracle.schatten(colmajor(G, 30), 30, 17, 30, p))
        assert abs(got - s1) <= 200 * EPS * s1, p
    d = rng.uniform(-4, 4, 12)
    D = np.diag(d)
    for p in (1.0, 1.5, 4.0):
        got = float(oracle.schatten(colmajor(D, 12), 12, 12, 12, p))
        want = float(np.sum(np.abs(d) ** p) ** (1 / p))
        assert abs(got - want) <= 100 * EPS * want, p


def test_nuclear_norm_of_2x2():
    rng = np.random.default_rng(2)
    for _ in range(50):
        a, b, c, d = rng.standard_normal(4)
        s1 = math.hypot(a + d, b - c)
        s2 = math.hypot(a - d, b + c)
        G = np.array([[a, b], [c, d]])
        got = float(oracle.schatten(colmajor(G, 2), 2, 2, 2, 1.0))
        assert abs(got - max(s1, s2)) <= 20 * EPS * max(s1, s2)


def test_orthogonal_invariance():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((25, 18))
    Q, _ = np.linalg.qr(rng.standard_normal((25, 25)))
    for p in (1.0, 3.0, math.inf):
        a = float(oracle.schatten(colmajor(G, 25), 25, 18, 25, p))
        b = float(oracle.schatten(colmajor(Q @ G, 25), 25, 18, 25, p))
        assert abs(a - b) <= 500 * EPS * a, p
