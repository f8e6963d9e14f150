"""Complex vectors on the GPU: the real-view tree (bitwise the real call on 2n elements for
unit stride, and the contiguous copy's bits for any stride), parity with the oracle,
special values and argument errors."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, bits, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

SIZES = [1, 2, 3, 63, 64, 65, 4095, 4096, 4097, 8193, 100003, (1 << 20) + 7]


def cvec(n, fmt, seed):
    r = vnp_gen.host_fill(2 * n, dtype=fmt, kind="exp", lo=-20, hi=20, seed=seed, stream=41)
    return r[0::2] + 1j * r[1::2] if fmt == "f64" else (r[0::2] + 1j * r[1::2]).astype(np.complex64)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_parity_and_real_view(fmt):
    for i, n in enumerate(SIZES):
        print(f"complex {fmt} n={n}", flush=True)
        z = cvec(n, fmt, i)
        zd = to_dev(z)
        g = vnp.nrmf_complex(zd).item()
        assert_parity(g, oracle.nrmf_complex(z), 2 * n, fmt, f"n={n}")
        view = torch.view_as_real(zd).reshape(-1)
        assert bits(g, fmt) == bits(vnp.nrmf(view).item(), fmt)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_strides_give_the_contiguous_bits(fmt):
    n = 50001
    for incz in (2, 3, -1, -4):
        z = cvec(n * abs(incz), fmt, 100 + abs(incz))
        sel = z[::abs(incz)][:n]
        if incz < 0:
            sel = sel[::-1]
        want = vnp.nrmf_complex(to_dev(np.ascontiguousarray(sel))).item()
        got = vnp.nrmf_complex(to_dev(z), n=n, incz=incz).item()
        print(f"complex {fmt} incz={incz}", flush=True)
        assert bits(got, fmt) == bits(want, fmt)
        assert_parity(got, oracle.nrmf_complex(z, incz=incz, n=n), 2 * n, fmt)


def test_special_values_and_errors():
    z = np.array([3 + 4j, 0j, 0j], dtype=np.complex128)
    assert vnp.nrmf_complex(to_dev(z)).item() == 5.0
    z[1] = complex(math.inf, 0)
    assert vnp.nrmf_complex(to_dev(z)).item() == math.inf
    z[2] = complex(0, math.nan)
    assert math.isnan(vnp.nrmf_complex(to_dev(z)).item())
    e = torch.zeros(0, dtype=torch.complex128, device="cuda")
    assert vnp.nrmf_complex(e, n=0).item() == 0.0
    L = vnp.lib()
    out = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.vnp_dznrmf(1 << 40, None, 1, out.data_ptr(), s) == -1
    assert L.vnp_dznrmf(3, None, 1, out.data_ptr(), s) == -2
    zz = to_dev(np.zeros(3, dtype=np.complex128))
    assert L.vnp_dznrmf(3, zz.data_ptr(), 0, out.data_ptr(), s) == -3
    assert L.vnp_dznrmf(3, zz.data_ptr(), 1, None, s) == -4
