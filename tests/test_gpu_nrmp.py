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


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", [0.25, 0.3, 0.5, 0.75, 1.5, 3.0, 4.5, 8.0, 100.0])
def test_pnode_accuracy(fmt, p):
    """The device p node on 4096 pairs spanning magnitude ratios 1 .. 2^-80 (as two-element
    segments, so each result is one leaf node) against the binary128 reference and the
    oracle's Listing 5 node with a correctly rounded pow.  Bounds: binary64 4 max(1, 1/p)
    eps (an absolute error in log2 Z reaches C multiplied by 1/p); binary32 (1.1 + ln2 / p)
    eps: the final rounding of the binary64 evaluation plus the binary32 rounding of the
    exponent 1/p, which the single-precision node uses (Sect. 4)."""
    rng = np.random.default_rng(int(p * 1000) + (1 if fmt == "f32" else 0))
    npairs = 4096
    a = np.ldexp(rng.uniform(0.5, 1.0, npairs), rng.integers(-30, 30, npairs))
    b = a * np.ldexp(rng.uniform(0.5, 1.0, npairs), -rng.integers(0, 80, npairs))
    b[:64] = a[:64]  # equal operands
    b[64:128] = np.nextafter(a[64:128], 0)
    x = np.empty(2 * npairs)
    x[0::2], x[1::2] = a, b
    sign = rng.random(2 * npairs) < 0.5
    x[sign] = -x[sign]
    npdt = np.float64 if fmt == "f64" else np.float32
    x = x.astype(npdt)
    off = np.arange(0, 2 * npairs + 1, 2, dtype=np.int64)
    g = vnp.nrm_batched(to_dev(x), to_dev(off), p=p).cpu().numpy().astype(np.float64)
    eps = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    worst_ref = worst_or = 0.0
    for i in range(npairs):
        pair = x[2 * i:2 * i + 2]
        hi, lo = oracle.ref_pnorm(pair, p)
        ref = hi + lo
        worst_ref = max(worst_ref, abs(g[i] - ref) / ref / eps)
        o = float(oracle.nrmp(pair, p, "A"))
        worst_or = max(worst_or, abs(g[i] - o) / o / eps)
    print(f"p={p} {fmt}: node error vs binary128 {worst_ref:.3f} eps, vs oracle node {worst_or:.3f} eps", flush=True)
    bound = 4.0 * max(1.0, 1.0 / p) if fmt == "f64" else 1.1 + math.log(2.0) / p
    assert worst_ref <= bound, (worst_ref, bound)
    assert worst_or <= 2 * bound + 1, (worst_or, bound)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_graph_capture_of_the_p_node(fmt):
    """The p node's per-p tables travel in the kernel arguments, so a captured call keeps
    them: every replay of a captured DNRMP (streaming and finish kernels, a ragged tail
    tile) equals the eager call, with calls at other p in between."""
    dt = torch.float64 if fmt == "f64" else torch.float32
    n = (1 << 21) + 321
    x = torch.empty(n, dtype=dt, device="cuda")
    out = torch.empty((), dtype=dt, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        vnp_gen.dev_fill(x, kind="exp", lo=-10, hi=10, seed=3)
        vnp.nrmp(x, 3.0, out=out)  # warm-up: the stream's workspace
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        vnp.nrmp(x, 3.0, out=out)
    for rep in range(4):
        vnp_gen.dev_fill(x, kind="exp", lo=-10, hi=10, seed=200 + rep)
        torch.cuda.synchronize()
        other = vnp.nrmp(x, 1.5 + rep).item()  # another p, eagerly, between replays
        eager = vnp.nrmp(x, 3.0).item()
        g.replay()
        torch.cuda.synchronize()
        assert out.item() == eager, rep
        assert other != eager


def test_many_distinct_p():
    """More distinct p values than the host keeps tables for (the cache is cleared and
    refilled): each result stays within the parity bar of the oracle's A_p."""
    rng = np.random.default_rng(17)
    x = vnp_gen.host_fill(3000, dtype="f64", kind="exp", lo=-5, hi=5, seed=9, stream=3)
    d = to_dev(x)
    for p in np.concatenate([rng.uniform(0.5, 20.0, 290), [0.5, 7.0]]):
        p = float(p)
        if p in (1.0, 2.0):
            continue
        g = gpu_p(d, p)
        o = float(oracle.nrmp(x, p, "A"))
        assert_parity(g, o, 3000, "f64")


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_pnorm_launch_shapes_are_bitwise_identical(fmt):
    """The p node gives the same bits in every launch shape (small-vector kernel, streaming
    kernel with a partial tail tile evaluated out of line, several shapes)."""
    te = 16384 if fmt == "f32" else 8192
    try:
        for n in [3 * te + 17, (1 << 20) + 12345]:
            x = to_dev(vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-10, hi=10, seed=8))
            ref = gpu_p(x, 3.0)
            for wpb, wt in [(1, 1), (4, 1), (4, 4), (8, 8), (16, 2)]:
                vnp.set_launch_shape(wpb, wt)
                assert gpu_p(x, 3.0) == ref, (n, wpb, wt)
            vnp.set_launch_shape(0, 0)
            assert gpu_p(x, 3.0) == ref
    finally:
        vnp.set_launch_shape(0, 0)


@pytest.mark.parametrize("p", [3.0, 0.5, 2.0 ** -20, 2.0 ** -21])
def test_pnode_row_classes(p):
    """Zeros, infinities, NaN and overflow through the binary64 row levels, which carry
    log2 of each partial norm (1/p <= 2^20) or the value itself (1/p > 2^20): zero runs
    stay exact, NaN beats inf wherever each one sits, an overflowing norm is +inf.  One
    nonzero element among zeros gives its magnitude (Sect. 4's node with Q = 0 is exact):
    bitwise in the value domain, and within the rounding of 2^l at the row root (2 eps) in
    the logarithmic one."""
    n = 3 * 8192 + 517  # several tiles and a ragged tail tile
    z = np.zeros(n)
    assert gpu_p(to_dev(z), p) == 0.0
    for i in [0, 1, 63, 4097, n - 1]:
        y = z.copy()
        y[i] = -1.2345e-300 if i % 2 else 6.5e305
        g = gpu_p(to_dev(y), p)
        if p < 2.0 ** -20:
            assert g == abs(y[i]), (p, i)
        else:
            assert abs(g - abs(y[i])) <= 2 * 2.0 ** -53 * abs(y[i]), (p, i, g)
    y = z.copy()
    y[[5, 9000]] = [1.5, -2.0]
    if p < 2.0 ** -19:  # |x|^p ~ 1 for both: (1 + 1)^(1/p) overflows
        assert gpu_p(to_dev(y), p) == math.inf
    else:
        assert_parity(gpu_p(to_dev(y), p), oracle.nrmp(y, p), n, "f64", f"p={p}")
    w = vnp_gen.host_fill(n, dtype="f64", kind="exp", lo=-10, hi=10, seed=21)
    w[::7] = 0.0
    v = w.copy()
    v[8191] = np.inf
    assert gpu_p(to_dev(v), p) == math.inf
    v[20000] = np.nan  # another tile than the infinity
    assert math.isnan(gpu_p(to_dev(v), p))
    v = w.copy()
    v[3] = np.nan
    v[n - 2] = -np.inf
    assert math.isnan(gpu_p(to_dev(v), p))
    big = np.full(4096, 1.0e308)
    assert gpu_p(to_dev(big), p) == math.inf
    if p >= 0.5:
        assert_parity(gpu_p(to_dev(w), p), oracle.nrmp(w, p), n, "f64", f"p={p}")
        sub = w * 1e-310  # subnormal elements and partial norms
        assert_parity(gpu_p(to_dev(sub), p), oracle.nrmp(sub, p), n, "f64", f"p={p} subnormal")


@pytest.mark.parametrize("p", [3.0, 0.5])
def test_pnode_row_classes_streamed(p):
    """The same classes through the streaming kernel (enough tiles for it; a ragged tail
    tile evaluated out of line) and through the batched kernel: zeros in whole row groups,
    an infinity or a NaN in a streamed tile and in the tail tile, and one nonzero element
    among zeros; each streamed result equals the batched one for the same segment."""
    te = 8192
    n = 1100 * te + 517  # above the small-vector limit of 4 tiles per CU (256 CUs)
    w = vnp_gen.host_fill(n, dtype="f64", kind="exp", lo=-10, hi=10, seed=31)
    w[1000:5000] = 0.0  # zero row groups inside a streamed tile
    w[n - 300:] = 0.0  # the tail tile ends in zeros
    cases = {"finite": w}
    v = w.copy(); v[777 * te + 4321] = np.inf; cases["inf streamed"] = v
    v = w.copy(); v[n - 400] = -np.inf; cases["inf tail"] = v
    v = w.copy(); v[5 * te + 1] = np.nan; v[n - 350] = np.inf; cases["nan streamed, inf tail"] = v
    v = w.copy(); v[n - 450] = np.nan; v[3] = np.inf; cases["inf streamed, nan tail"] = v
    z = np.zeros(n); z[600 * te + 77] = -3.25e-200; cases["one nonzero"] = z
    for name, x in cases.items():
        d = to_dev(x)
        g = gpu_p(d, p)
        off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
        gb = vnp.nrm_batched(d, off, p=p).item()
        print(f"p={p} {name}: {g!r} batched {gb!r}", flush=True)
        assert (math.isnan(g) and math.isnan(gb)) or g == gb, (name, g, gb)
        if name == "finite":
            assert_parity(g, oracle.nrmp(x, p), n, "f64", f"p={p} {name}")
        elif "nan" in name:
            assert math.isnan(g), name
        elif "inf" in name:
            assert g == math.inf, name
        else:
            assert abs(g - 3.25e-200) <= 2 * 2.0 ** -53 * 3.25e-200, (name, g)
