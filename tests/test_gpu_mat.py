"""Norm of a whole array with a leading dimension (Sect. 3.1) on the GPU: parity with the
oracle, the contiguous-array identity (bitwise the single-vector call), rows past m never
read, empty arrays and argument errors."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, bits, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

SHAPES = [(1, 10, 2), (3, 4097, 5), (1000, 37, 1003), (8192, 64, 8200), (8193, 5, 8200), (100000, 3, 100001),
          (20000, 300, 20011)]


def stored(m, ncols, lda, fmt, seed):
    a = vnp_gen.host_fill(lda * ncols, dtype=fmt, kind="exp", lo=-20, hi=20, seed=seed, stream=31)
    a2 = a.reshape(ncols, lda)
    a2[:, m:] = np.nan  # padding rows must never be read
    return a


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", [2.0, 1.0, 3.0, math.inf])
def test_parity_against_oracle(fmt, p):
    for i, (m, ncols, lda) in enumerate(SHAPES):
        print(f"mat {fmt} p={p} m={m} ncols={ncols} lda={lda}", flush=True)
        a = stored(m, ncols, lda, fmt, i)
        g = vnp.nrm_mat(to_dev(a), m, ncols, lda, p=p).item()
        o = oracle.nrm_mat(a, m, ncols, lda, p=p)
        assert not math.isnan(g)
        if p == math.inf:
            assert g == o  # the max node is exact
        else:
            # column trees and the tree over columns: at most one level deeper than a tree
            # over m ncols elements
            assert_parity(g, o, 2 * m * ncols, fmt, f"m={m} ncols={ncols}")


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_contiguous_array_is_one_vector(fmt):
    m, ncols = 1000, 777
    a = to_dev(vnp_gen.host_fill(m * ncols, dtype=fmt, kind="exp", lo=-20, hi=20, seed=4))
    for p in (2.0, 3.0):
        g = vnp.nrm_mat(a, m, ncols, m, p=p).item()
        ref = (vnp.nrmf(a) if p == 2.0 else vnp.nrmp(a, p)).item()
        assert bits(g, fmt) == bits(ref, fmt)
    col = vnp.nrm_mat(a, m, 1, m + 50).item()  # one column
    assert bits(col, fmt) == bits(vnp.nrmf(a[:m]).item(), fmt)


def test_empty_and_argument_errors():
    a = torch.zeros(100, dtype=torch.float64, device="cuda")
    assert vnp.nrm_mat(a, 0, 5, 1).item() == 0.0
    assert vnp.nrm_mat(a, 5, 0, 5).item() == 0.0
    L = vnp.lib()
    out = torch.empty((), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.vnp_dnrmf_mat(-1, 2, a.data_ptr(), 1, out.data_ptr(), s) == -1
    assert L.vnp_dnrmf_mat(2, -1, a.data_ptr(), 2, out.data_ptr(), s) == -2
    assert L.vnp_dnrmf_mat(2, 2, None, 2, out.data_ptr(), s) == -3
    assert L.vnp_dnrmf_mat(4, 2, a.data_ptr(), 3, out.data_ptr(), s) == -4
    assert L.vnp_dnrmf_mat(2, 2, a.data_ptr(), 2, None, s) == -5
    assert L.vnp_dnrmp_mat(2, 2, a.data_ptr(), 2, 0.0, out.data_ptr(), s) == -5
    assert L.vnp_dnrmp_mat(2, 2, a.data_ptr(), 2, 3.0, None, s) == -6
    assert L.vnp_dnrmf_mat(1 << 21, 1 << 20, a.data_ptr(), 1 << 21, out.data_ptr(), s) == -4  # > 2^40 elements
