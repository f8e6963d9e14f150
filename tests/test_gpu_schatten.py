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

SHAPES = [(8, 8, 8), (37, 20, 40), (20, 37, 20), (100, 64, 128), (200, 200, 201)]


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
