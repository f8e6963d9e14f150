"""GPU parity for the p-norm: the HIP tree with the Listing-5 node against the oracle's A_p."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

PS = [1.0, 1.5, 3.0, 4.5, 8.0, math.inf, 2.0 ** 60, 0.5, math.sqrt(2), math.e, math.pi]
SIZES = [1, 2, 3, 7, 64, 129, 1000, 8193, (1 << 16) + 3, (1 << 20) + 1]


def gpu_p(x, p, n=None, incx=1):
    out = vnp.nrmp(x, p, n=n, incx=incx)
    torch.cuda.synchronize()
    return out.item()


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", PS)
def test_pnorm_parity(fmt, p):
    for i, n in enumerate(SIZES):
        x = vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-10, hi=10, seed=i, stream=5)
        print(f"pnorm {fmt} p={p} n={n}", flush=True)
        g = gpu_p(to_dev(x), p)
        o = oracle.nrmp(x, p)
        if math.isinf(p) or p >= 2 ** 53:
            assert g == float(np.abs(x).max())
        assert_parity(g, o, n, fmt, f"p={p} n={n}")
    assert oracle.counters()["pow_unresolved"] == 0


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_p2_is_the_frobenius_norm(fmt):
    x = to_dev(vnp_gen.host_fill(100003, dtype=fmt, kind="exp", lo=-10, hi=10, seed=3))
    assert gpu_p(x, 2.0) == vnp.nrmf(x).item()
    # a p next to 2 goes through the generic node and stays within the tolerance of NRMF
    xs = x.cpu().numpy()
    assert_parity(gpu_p(x, 2.0000001), oracle.nrmp(xs, 2.0000001), xs.size, "f64" if fmt == "f64" else "f32")


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_pnorm_strides_and_specials(fmt):
    n = 50001
    x = vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-10, hi=10, seed=8)
    ref = gpu_p(to_dev(x), 3.0)
    buf = np.zeros(2 * n - 1, dtype=x.dtype)
    buf[::2] = x
    assert gpu_p(to_dev(buf), 3.0, n=n, incx=2) == ref
    y = x.copy()
    y[100] = np.nan
    assert math.isnan(gpu_p(to_dev(y), 3.0))
    y[100] = np.inf
    assert gpu_p(to_dev(y), 3.0) == math.inf
    assert gpu_p(to_dev(y), 1.0) == math.inf
    assert gpu_p(to_dev(y), math.inf) == math.inf
    ints = np.arange(-300, 301, dtype=x.dtype)
    assert gpu_p(to_dev(ints), 1.0) == float(np.abs(ints).sum())
