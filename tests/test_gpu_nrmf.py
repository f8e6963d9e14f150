"""GPU parity: the HIP single-vector norms against the CPU oracle (A: R with cr_hypot),
bitwise reproducibility across launch shapes, alignment and strides, and special values."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, bits, fmt_of, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

TD, TS = 8192, 16384
SIZES = [1, 2, 3, 4, 5, 7, 8, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 4095, 8191, 8192, 8193, 16383,
         16384, 16385, 3 * 8192 + 17, 65536 + 5, 1 << 20, (1 << 20) + 12345]
DISTS = [("u11", 0, 0), ("exp", -20, 20), ("exp", -300, 300)]


def gpu_norm(x, n=None, incx=1):
    out = vnp.nrmf(x, n=n, incx=incx)
    torch.cuda.synchronize()
    return out.item()


@pytest.fixture(autouse=True)
def _reset_shape():
    vnp.set_launch_shape(0, 0)
    yield
    vnp.set_launch_shape(0, 0)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("dist", DISTS)
def test_parity_against_oracle(fmt, dist):
    kind, lo, hi = dist
    for i, n in enumerate(SIZES):
        x = vnp_gen.host_fill(n, dtype=fmt, kind=kind, lo=lo, hi=hi, seed=i, stream=3)
        print(f"parity {fmt} {kind}[{lo},{hi}] n={n}", flush=True)
        g = gpu_norm(to_dev(x))
        assert_parity(g, oracle.nrmf(x, "A"), n, fmt, f"n={n}")


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_empty_and_single(fmt):
    dt = torch.float64 if fmt == "f64" else torch.float32
    assert vnp.nrmf(torch.zeros(0, dtype=dt, device="cuda"), n=0).item() == 0.0
    assert vnp.nrmf(torch.tensor([-2.5], dtype=dt, device="cuda")).item() == 2.5
    assert vnp.nrmf(torch.zeros(10000, dtype=dt, device="cuda")).item() == 0.0
    x = torch.tensor([3.0, -4.0], dtype=dt, device="cuda")
    assert vnp.nrmf(x).item() == 5.0


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_launch_shapes_are_bitwise_identical(fmt):
    for n in [3 * (TS if fmt == "f32" else TD) + 17, (1 << 20) + 12345]:
        x = to_dev(vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-20, hi=20, seed=7))
        ref = gpu_norm(x)
        for wpb, wt in [(1, 1), (2, 1), (4, 1), (4, 2), (4, 4), (8, 8), (16, 8), (16, 1), (1, 8)]:
            vnp.set_launch_shape(wpb, wt)
            print(f"shape {fmt} n={n} wpb={wpb} wt={wt}", flush=True)
            assert gpu_norm(x) == ref, (wpb, wt)
        vnp.set_launch_shape(0, 0)
        for _ in range(20):
            assert gpu_norm(x) == ref


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_one_hundred_reruns_are_bitwise_identical(fmt):
    """100 back-to-back calls on one stream (results kept on the device, one sync at the
    end) give the same bits, for a small vector (one block per tile) and one large enough
    for the streaming kernel and its finish launch."""
    for n, seed in ((1 << 20) + 7, 31), ((3 << 22) + 12345, 32):
        x = torch.empty(n, dtype=torch.float64 if fmt == "f64" else torch.float32, device="cuda")
        vnp_gen.dev_fill(x, kind="exp", lo=-20, hi=20, seed=seed)
        outs = torch.empty(100, dtype=x.dtype, device="cuda")
        for r in range(100):
            vnp.nrmf(x, out=outs[r])
        torch.cuda.synchronize()
        o = outs.cpu().numpy()
        u = o.view(np.uint64 if fmt == "f64" else np.uint32)
        assert np.all(u == u[0]), (n, np.unique(o))


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_longest_runs_per_wave(fmt):
    """Waves covering the maximum run of 2^12 tiles (all of it, and a ragged part) give
    the default shape's bits."""
    n = 4096 * (TS if fmt == "f32" else TD) + 12345
    xh = vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-20, hi=20, seed=17)
    x = to_dev(xh)
    ref = gpu_norm(x)
    assert_parity(ref, oracle.nrmf(xh, "A"), n, fmt)
    for wpb, wt in ((1, 4096), (2, 4096), (16, 4096), (4, 2048)):
        print(f"{fmt} n={n} shape ({wpb}, {wt})", flush=True)
        vnp.set_launch_shape(wpb, wt)
        assert bits(gpu_norm(x), fmt) == bits(ref, fmt), (wpb, wt)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_alignment_and_strides_are_bitwise_identical(fmt):
    n = (1 << 18) + 333
    x = vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=-20, hi=20, seed=9)
    ref = gpu_norm(to_dev(x))
    for off in (1, 2, 3):
        buf = np.zeros(n + off, dtype=x.dtype)
        buf[off:] = x
        d = to_dev(buf)
        print(f"offset {fmt} {off}", flush=True)
        assert gpu_norm(d[off:], n=n) == ref
    for inc in (2, 3, -1, -4):
        a = abs(inc)
        buf = np.full((n - 1) * a + 1, np.nan, dtype=x.dtype)
        buf[::a] = x if inc > 0 else x[::-1]
        print(f"stride {fmt} {inc}", flush=True)
        assert gpu_norm(to_dev(buf), n=n, incx=inc) == ref


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_special_values(fmt):
    dt = np.float64 if fmt == "f64" else np.float32
    for n, pos in [(5, 2), (100000, 77777), (3 * 16384 + 5, 3 * 16384 + 1)]:
        base = vnp_gen.host_fill(n, dtype=fmt, kind="u11", seed=1)
        for vals, want in [([np.nan], "nan"), ([np.inf], "inf"), ([-np.inf], "inf"), ([np.inf, np.nan], "nan")]:
            x = base.copy()
            for j, v in enumerate(vals):
                x[(pos + 13 * j) % n] = v
            g = gpu_norm(to_dev(x))
            assert (math.isnan(g) if want == "nan" else g == math.inf), (n, vals, g)
            o = oracle.nrmf(x, "A")
            assert (math.isnan(o) if want == "nan" else o == math.inf)
    big = np.finfo(dt).max
    assert gpu_norm(to_dev(np.array([big, big], dtype=dt))) == math.inf
    assert gpu_norm(to_dev(np.array([big / 2, big / 2], dtype=dt))) < math.inf
    assert gpu_norm(to_dev(np.array([big, 1.0], dtype=dt))) == big
    tiny = np.float64(2.0 ** -1074) if fmt == "f64" else np.float32(2.0 ** -149)
    assert gpu_norm(to_dev(np.array([3 * tiny, 4 * tiny], dtype=dt))) == 5 * tiny


def _f32_cases():
    """binary32 inputs for the streamed tiles' finite-operand node and its NaN-root fallback:
    zero pairs and sparse vectors, the subnormal and near-overflow ranges, an overflow
    inside one tile, and infinities and NaNs in single tiles."""
    n = 5 * 16384 + 333
    big = np.float32(np.finfo(np.float32).max)
    out = []
    x = vnp_gen.host_fill(n, dtype="f32", kind="u11", seed=21)
    x[np.arange(n) % 10 != 3] = 0.0  # 90% zeros: many (0, 0) leaves and zero subtrees
    out.append(("sparse", x))
    x = np.zeros(n, dtype=np.float32)
    x[4 * 16384 + 7] = -3.0
    out.append(("one nonzero", x))
    out.append(("exp[-149,-100]", vnp_gen.host_fill(n, dtype="f32", kind="exp", lo=-149, hi=-100, seed=22)))
    out.append(("exp[-149,60]", vnp_gen.host_fill(n, dtype="f32", kind="exp", lo=-149, hi=60, seed=23)))
    out.append(("exp[90,126]", vnp_gen.host_fill(n, dtype="f32", kind="exp", lo=90, hi=126, seed=24)))
    x = vnp_gen.host_fill(n, dtype="f32", kind="u11", seed=25)
    x[2 * 16384 + 100] = big
    x[2 * 16384 + 101] = big  # the pair overflows to +inf inside tile 2
    out.append(("overflow in a tile", x))
    x = vnp_gen.host_fill(n, dtype="f32", kind="u11", seed=26)
    x[3 * 16384 - 1] = big
    x[3 * 16384] = -big  # near-overflow values in two tiles, each tile root finite
    out.append(("big in two tiles", x))
    for v, name in [(np.inf, "inf"), (-np.inf, "-inf"), (np.nan, "nan")]:
        for pos in (0, 16384 + 5, n - 1):
            x = vnp_gen.host_fill(n, dtype="f32", kind="u11", seed=27)
            x[pos] = v
            out.append((f"{name} at {pos}", x))
    x = vnp_gen.host_fill(n, dtype="f32", kind="u11", seed=28)
    x[100], x[4 * 16384 + 9] = np.inf, np.nan
    out.append(("inf and nan", x))
    return out


def test_f32_streamed_tiles_match_the_guarded_node():
    """The streamed binary32 tiles use a node without the special-value guard and fall back
    to the guarded node for a wave whose tile root is NaN; the small-vector kernel uses the
    guarded node throughout.  The forced launch shapes (streamed tiles) must give the
    small-vector kernel's bits on every case, and the oracle's value within the bound."""
    for name, x in _f32_cases():
        d = to_dev(x)
        vnp.set_launch_shape(0, 0)
        ref = gpu_norm(d)  # small vector: one block per tile, guarded node
        o = oracle.nrmf(x, "A")
        print(f"f32 streamed vs guarded: {name}: {ref!r} (oracle {o!r})", flush=True)
        assert_parity(ref, o, x.size, "f32", name)
        for wpb, wt in [(1, 1), (4, 2), (1, 8), (16, 1)]:
            vnp.set_launch_shape(wpb, wt)
            g = gpu_norm(d)
            assert bits(g, "f32") == bits(ref, "f32") or (math.isnan(g) and math.isnan(ref)), (name, wpb, wt, g, ref)
        vnp.set_launch_shape(0, 0)


@pytest.mark.parametrize("fmt,lo,hi,expect_inf", [("f64", 990, 1023, True), ("f64", 990, 1007, False),
                                                  ("f64", -1074, -1000, False), ("f32", 94, 127, True),
                                                  ("f32", -149, -104, False)])
def test_stress_ranges(fmt, lo, hi, expect_inf):
    n = (1 << 22) + 7
    x = vnp_gen.host_fill(n, dtype=fmt, kind="exp", lo=lo, hi=hi, seed=2)
    g = gpu_norm(to_dev(x))
    o = oracle.nrmf(x, "A")
    if expect_inf:
        assert g == math.inf and o == math.inf
    else:
        assert math.isfinite(g)
        assert_parity(g, o, n, fmt)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_accuracy_against_exact(fmt):
    # Sect. 2 reports relative errors below 3 eps for the recursive algorithms on such data.
    n = 1 << 22
    x = vnp_gen.host_fill(n, dtype=fmt, kind="u01", seed=4)
    g = gpu_norm(to_dev(x))
    e = oracle.exact_nrm2(x)
    assert oracle.relerr(g, e, fmt) < 3.0


def test_invalid_arguments():
    L = vnp.lib()
    assert L.vnp_dnrmf(10, 0, 1, 0, None) == -2
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert L.vnp_dnrmf(4, x.data_ptr(), 0, x.data_ptr(), None) == -3
    assert L.vnp_dnrmf(4, x.data_ptr(), 1, 0, None) == -4
    assert L.vnp_dnrmp(4, x.data_ptr(), 1, -1.0, x.data_ptr(), None) == -4
    assert L.vnp_dnrmp(4, x.data_ptr(), 1, float("nan"), x.data_ptr(), None) == -4
    assert L.vnp_dnrmf((1 << 40) + 1, x.data_ptr(), 1, x.data_ptr(), None) == -1


def test_concurrent_streams_from_threads():
    """Plain calls from four host threads on four streams (one workspace per stream): every
    result bitwise equal to the sequential one."""
    import threading

    xs = [to_dev(vnp_gen.host_fill(n, kind="exp", lo=-20, hi=20, seed=60 + i))
          for i, n in enumerate((1 << 20, 3 * 8192 + 5, (1 << 22) + 17, 777))]
    ref = [gpu_norm(x) for x in xs]
    streams = [torch.cuda.Stream() for _ in xs]
    got = [[None] * 20 for _ in xs]

    def work(i):
        with torch.cuda.stream(streams[i]):
            outs = [vnp.nrmf(xs[i]) for _ in range(20)]
            streams[i].synchronize()
            got[i] = [o.item() for o in outs]

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(xs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, r in enumerate(ref):
        assert all(bits(g, "f64") == bits(r, "f64") for g in got[i]), i


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_graph_capture_and_replay(fmt):
    """A plain call captured in a HIP graph (after a warm-up call on the capture stream, so
    its workspace exists): every replay, with new data and eager work between replays,
    equals the eager call on the same data."""
    dt = torch.float64 if fmt == "f64" else torch.float32
    n = (1 << 21) + 123
    x = torch.empty(n, dtype=dt, device="cuda")
    out = torch.empty((), dtype=dt, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        vnp_gen.dev_fill(x, kind="exp", lo=-20, hi=20, seed=1)
        vnp.nrmf(x, out=out)  # warm-up: creates the stream's workspace
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        vnp.nrmf(x, out=out)
    for rep in range(5):
        vnp_gen.dev_fill(x, kind="exp", lo=-20, hi=20, seed=100 + rep)
        torch.cuda.synchronize()
        eager = vnp.nrmf(x).item()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert bits(out.item(), fmt) == bits(eager, fmt), rep
