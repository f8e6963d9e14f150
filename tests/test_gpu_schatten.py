"""Schatten p-norm on the GPU (rocSOLVER singular values, the library's p-norm) against the
oracle (LAPACK singular values, A_p).  The two SVDs differ by their backward errors:
singular values carry absolute errors of order max(m, n) eps sigma_1, so the tolerance is
4 k^(1/p) max(m, n) eps (k = min(m, n)) plus the tree's 2 (ceil(log2 k) + 1) eps."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

SHAPES = [(8, 8, 8), (37, 20, 40), (20, 37, 20), (100, 64, 128), (200, 200, 201), (700, 450, 704)]


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", [1.0, 2.0, 3.0, math.inf])
def test_parity_against_oracle(fmt, p):
    dt = np.float64 if fmt == "f64" else np.float32
    eps = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    for i, (m, n, lda) in enumerate(SHAPES):
        G = np.random.default_rng(10 * i + int(p if p < 10 else 9)).standard_normal((m, n))
        a = np.full(lda * n, np.nan, dtype=dt)
        for j in range(n):
            a[j * lda:j * lda + m] = G[:, j]
        g = vnp.schatten(to_dev(a), m, n, lda, p).item()
        o = float(oracle.schatten(a, m, n, lda, p))
        k = min(m, n)
        kp = k if p == 1.0 else (1.0 if p == math.inf else k ** (1.0 / p))
        tol = (4 * kp * max(m, n) + 2 * (math.ceil(math.log2(k)) + 1)) * eps
        print(f"schatten {fmt} p={p} {m}x{n}: rel diff {abs(g - o) / o:.3e} (tol {tol:.3e})", flush=True)
        assert abs(g - o) <= tol * o


@pytest.mark.parametrize("p", [1.0, 2.0, 3.0, math.inf])
def test_graded_singular_values(p):
    """G = U diag(s) V^T with s_i from 1 down to 1e-12 (random orthogonal U, V): the GPU and
    oracle norms agree within the same tolerance, and both within it of the norm of s."""
    rng = np.random.default_rng(77)
    m, n = 300, 240
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -12, n)
    G = (U * s) @ V.T
    a = np.asfortranarray(G).reshape(-1, order="F").copy()
    g = vnp.schatten(to_dev(a), m, n, m, p).item()
    o = float(oracle.schatten(a, m, n, m, p))
    exact = float(np.max(s)) if p == math.inf else float(np.sum(s ** p) ** (1.0 / p))
    kp = n if p == 1.0 else (1.0 if p == math.inf else n ** (1.0 / p))
    tol = (4 * kp * m + 2 * (math.ceil(math.log2(n)) + 1)) * 2.0 ** -53
    print(f"graded p={p}: gpu {abs(g - exact) / exact:.3e}, oracle {abs(o - exact) / exact:.3e} (tol {tol:.3e})",
          flush=True)
    assert abs(g - o) <= tol * o
    assert abs(g - exact) <= tol * exact


def test_special_cases_and_errors():
    z = torch.zeros(16, dtype=torch.float64, device="cuda")
    assert vnp.schatten(z, 0, 4, 1, 2.0).item() == 0.0
    assert vnp.schatten(z, 4, 4, 4, 3.0).item() == 0.0  # zero matrix
    d = np.diag([3.0, -4.0]).T.ravel()  # column-major 2 x 2
    assert abs(vnp.schatten(to_dev(d), 2, 2, 2, 2.0).item() - 5.0) <= 1e-15 * 5
    assert abs(vnp.schatten(to_dev(d), 2, 2, 2, math.inf).item() - 4.0) <= 1e-15 * 4
    L = vnp.lib()
    out = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.vnp_dschatten(-1, 2, z.data_ptr(), 1, 2.0, out.data_ptr(), s) == -1
    assert L.vnp_dschatten(2, -1, z.data_ptr(), 2, 2.0, out.data_ptr(), s) == -2
    assert L.vnp_dschatten(2, 2, None, 2, 2.0, out.data_ptr(), s) == -3
    assert L.vnp_dschatten(4, 2, z.data_ptr(), 3, 2.0, out.data_ptr(), s) == -4
    assert L.vnp_dschatten(2, 2, z.data_ptr(), 2, -1.0, out.data_ptr(), s) == -5
    assert L.vnp_dschatten(2, 2, z.data_ptr(), 2, 2.0, None, s) == -6


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_rank_deficient_scaled_and_vectors(fmt):
    """Rank-deficient matrices (zero singular values), entries near the ends of the exponent
    range (the off-diagonal scaling), and k = 1 (a row or a column: the Euclidean norm)."""
    dt = np.float64 if fmt == "f64" else np.float32
    eps = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    rng = np.random.default_rng(5)
    m, n, r = 120, 90, 30
    G = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))  # rank 30
    big, tiny = (2.0 ** 900, 2.0 ** -900) if fmt == "f64" else (2.0 ** 100, 2.0 ** -100)
    for scale in (1.0, big, tiny):
        a = np.asfortranarray(G * scale).reshape(-1, order="F").astype(dt)
        for p in (1.0, 2.0, 3.0, math.inf):
            g = vnp.schatten(to_dev(a), m, n, m, p).item()
            o = float(oracle.schatten(a, m, n, m, p))
            kp = n if p == 1.0 else (1.0 if p == math.inf else n ** (1.0 / p))
            tol = (4 * kp * m + 2 * (math.ceil(math.log2(n)) + 1)) * eps
            print(f"rank-30 {fmt} scale 2^{math.log2(scale):.0f} p={p}: rel diff {abs(g - o) / o:.3e}", flush=True)
            assert abs(g - o) <= tol * o
    v = rng.standard_normal(333).astype(dt)
    want = float(oracle.nrmf(v))
    for m_, n_ in ((333, 1), (1, 333)):
        g = vnp.schatten(to_dev(v), m_, n_, m_, 1.0).item()
        assert abs(g - want) <= 4 * eps * want


def test_non_finite_entries_give_nan():
    a = np.random.default_rng(9).standard_normal(16 * 12)
    for bad in (np.nan, np.inf):
        b = a.copy()
        b[37] = bad
        assert math.isnan(vnp.schatten(to_dev(b), 16, 12, 16, 1.0).item())
