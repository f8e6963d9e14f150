"""Input generator: the numpy definition and the C implementation agree bit for bit."""
import numpy as np
import pytest

import vnp_gen

CASES = [("u11", 0, 0), ("exp", -20, 20), ("exp", 990, 1023), ("exp", -1074, -1000), ("u11exp", -30, 30),
         ("u01", 0, 0), ("exp", -149, -104), ("exp", 94, 127)]


def _bits(a):
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


@pytest.mark.parametrize("kind,lo,hi", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_numpy_matches_c(kind, lo, hi, dtype):
    a = vnp_gen.np_fill(20000, dtype=dtype, kind=kind, lo=lo, hi=hi, seed=5, stream=3, i0=12345)
    b = vnp_gen.host_fill(20000, dtype=dtype, kind=kind, lo=lo, hi=hi, seed=5, stream=3, i0=12345)
    assert np.array_equal(_bits(a), _bits(b))


def test_raw_draws_match_splitmix64_definition():
    # SplitMix64 started at state K: output i = mix(K + (i + 1) * GAMMA).
    k = vnp_gen.key(0, 0)
    m1, m2, mask = 0xBF58476D1CE4E5B9, 0x94D049BB133111EB, (1 << 64) - 1
    state, ref = k, []
    for _ in range(8):
        state = (state + vnp_gen.GAMMA) & mask
        z = state
        z = ((z ^ (z >> 30)) * m1) & mask
        z = ((z ^ (z >> 27)) * m2) & mask
        ref.append(z ^ (z >> 31))
    assert [int(v) for v in vnp_gen.np_draws(8, 0, 0, 0)] == ref
    assert [int(v) for v in vnp_gen.host_draws(8, 0, 0, 0)] == ref


def test_offsets_are_global_indices():
    full = vnp_gen.np_fill(1000, kind="exp", lo=-3, hi=3, seed=9)
    part = vnp_gen.np_fill(300, kind="exp", lo=-3, hi=3, seed=9, i0=500)
    assert np.array_equal(full[500:800], part)


def test_distribution_shapes():
    x = vnp_gen.host_fill(1 << 16, kind="exp", lo=-20, hi=20)
    m, e = np.frexp(np.abs(x))
    assert np.all((m >= 0.5) & (m < 1.0))
    assert set(np.unique(e)) == set(range(-20, 21))
    assert 0.45 < np.mean(x < 0) < 0.55
    u = vnp_gen.host_fill(1 << 16, kind="u11")
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.02
    s = vnp_gen.host_fill(1 << 14, kind="exp", lo=-1074, hi=-1000)
    assert np.all(s != 0) and np.any(np.abs(s) < 2.0 ** -1022)


def test_lengths_log_uniform():
    L = vnp_gen.log_uniform_lengths(8192, 0, 20, seed=0)
    assert L.min() >= 1 and L.max() < (1 << 20)
    lg = np.log2(L)
    assert 9.0 < lg.mean() < 10.5
