"""Helpers shared by the GPU tests (device buffers, comparisons against the oracle)."""
import math

import numpy as np

from oracle import bounds

TINY_D = 2.0 ** -1074
TINY_S = 2.0 ** -149


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fmt_of(a):
    return "f32" if a.dtype == np.float32 else "f64"


def assert_parity(g, o, n, fmt, note=""):
    """|G - O| <= 2 (ceil(log2 n) + 1) eps |O|, plus (K + 1) times the subnormal spacing
    (inexact underflow voids relative bounds); special values must match exactly."""
    g, o = float(g), float(o)
    if math.isnan(o) or math.isnan(g):
        assert math.isnan(o) and math.isnan(g), (g, o, note)
        return
    if math.isinf(o) or math.isinf(g):
        assert g == o, (g, o, note)
        return
    tol = bounds.tol_parity(n, fmt)
    k = 0 if n <= 1 else math.ceil(math.log2(n))
    absf = (k + 1) * (TINY_S if fmt == "f32" else TINY_D)
    assert abs(g - o) <= tol * abs(o) + absf, (g, o, (g - o) / o if o else None, note)


def bits(v, fmt):
    return np.array([v], dtype=np.float32 if fmt == "f32" else np.float64).view(
        np.uint32 if fmt == "f32" else np.uint64)[0]
