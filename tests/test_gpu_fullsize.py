"""Parity at the benchmark sizes, in the launch configuration the benchmark times.

One vector of n = 2^30 (binary64 and binary32; the plain range and the overflow-prone,
large finite and subnormal ranges) against the oracle (A: R with the correctly rounded
hypot) and the exact norm; the device-generated input is checked to be the host input.
p-norms at n = 2^28 against the binary128 reference, against the oracle where its node
is cheap (p = 1), exact power-of-two scaling, and p = 2 against the Frobenius call.
The oracle's A_p with a correctly rounded pow per node needs minutes at n = 2^28, so
the other p are pinned to it on the first 2^24 elements of the same recipe."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")

C1_CASES = [("f64", "c1", False), ("f64", "c1_overflow_d", True), ("f64", "c1_bigfinite_d", False),
            ("f64", "c1_subnormal_d", False), ("f32", "c1", False), ("f32", "c1_overflow_s", True),
            ("f32", "c1_subnormal_s", False)]


@pytest.fixture(autouse=True)
def _default_shape():
    vnp.set_launch_shape(0, 0)
    yield
    vnp.set_launch_shape(0, 0)
    torch.cuda.empty_cache()


def inputs(fmt, rec):
    r = vnp_gen.recipe(rec)
    n = r["n"]
    dt = torch.float64 if fmt == "f64" else torch.float32
    xd = torch.empty(n, dtype=dt, device="cuda")
    vnp_gen.dev_fill(xd, kind=r["kind"], lo=r["lo"], hi=r["hi"], seed=r["seed"], stream=r["stream"])
    xh = vnp_gen.host_fill(n, dtype=fmt, kind=r["kind"], lo=r["lo"], hi=r["hi"], seed=r["seed"], stream=r["stream"])
    idx = np.unique(np.concatenate([np.linspace(0, n - 1, 8193).astype(np.int64), np.arange(n - 64, n)]))
    got = xd[torch.from_numpy(idx).cuda()].cpu().numpy()
    ui = np.uint64 if fmt == "f64" else np.uint32
    assert np.array_equal(got.view(ui), xh[idx].view(ui)), "device generator differs from the host generator"
    return xd, xh


def eps(fmt):
    return 2.0 ** -53 if fmt == "f64" else 2.0 ** -24


@pytest.mark.parametrize("fmt,rec,overflows", C1_CASES)
def test_c1_full_size(fmt, rec, overflows):
    print(f"full size {fmt} {rec}", flush=True)
    xd, xh = inputs(fmt, rec)
    n = xh.size
    g = vnp.nrmf(xd).item()
    o = oracle.nrmf(xh, "A")
    if overflows:
        assert g == math.inf and o == math.inf, (g, o)
        return
    assert_parity(g, o, n, fmt, rec)
    ex = oracle.exact_nrm2(xh)
    print(f"  {rec} {fmt}: GPU {g!r}, oracle {o!r}, exact {ex!r}; error vs exact: GPU "
          f"{abs(g - ex) / ex / eps(fmt):.3f} eps, oracle {abs(o - ex) / ex / eps(fmt):.3f} eps", flush=True)
    if rec == "c1":
        # the same bits from other launch shapes (waves per block, tiles per wave)
        for wpb, wt in ((1, 1), (4, 8), (16, 4096)):
            vnp.set_launch_shape(wpb, wt)
            assert bits(vnp.nrmf(xd).item(), fmt) == bits(g, fmt), (wpb, wt)
        vnp.set_launch_shape(0, 0)


@pytest.mark.parametrize("p", [1.0, 1.5, 3.0, 4.5, 8.0])
def test_c2_full_size(p):
    print(f"full size p-norm p={p}", flush=True)
    xd, xh = inputs("f64", "c2")
    n = xh.size
    g = vnp.nrmp(xd, p).item()
    hi, lo = oracle.ref_pnorm(xh, p)
    ref = hi + lo
    tol = 2 * (math.ceil(math.log2(n)) + 1) * eps("f64")
    assert abs(g - ref) <= tol * ref, (g, ref, (g - ref) / ref / eps("f64"))
    print(f"  p={p}: GPU error vs binary128 reference {abs(g - ref) / ref / eps('f64'):.3f} eps", flush=True)
    if p == 1.0:
        assert_parity(g, oracle.nrmp(xh, 1.0, "A"), n, "f64", "p=1")
    # exact power-of-two scaling (no node crosses the subnormal or overflow range)
    xd.mul_(32.0)
    assert bits(vnp.nrmp(xd, p).item(), "f64") == bits(32.0 * g, "f64")


@pytest.mark.parametrize("p", [1.5, 3.0, 4.5, 8.0])
def test_c2_recipe_against_the_oracle_at_2p24(p):
    """A_p (the recursion with Listing 5's node and a correctly rounded pow) on the first
    2^24 elements of the C2 vector: the streaming kernel with runs of several tiles per
    wave, within the parity bound; and the binary128 reference for both."""
    r = vnp_gen.recipe("c2")
    n = 1 << 24
    xh = vnp_gen.host_fill(n, dtype="f64", kind=r["kind"], lo=r["lo"], hi=r["hi"], seed=r["seed"],
                           stream=r["stream"])
    xd = torch.from_numpy(xh).cuda()
    print(f"C2 recipe p={p} at 2^24 against A_p", flush=True)
    g = vnp.nrmp(xd, p).item()
    o = float(oracle.nrmp(xh, p, "A"))
    assert_parity(g, o, n, "f64", f"p={p}")
    hi, lo = oracle.ref_pnorm(xh, p)
    ref = hi + lo
    print(f"  p={p}: GPU {abs(g - ref) / ref / eps('f64'):.3f} eps, A_p {abs(o - ref) / ref / eps('f64'):.3f} eps "
          "from the binary128 reference", flush=True)


def test_c2_p2_is_frobenius():
    xd, _ = inputs("f64", "c2")
    assert bits(vnp.nrmp(xd, 2.0).item(), "f64") == bits(vnp.nrmf(xd).item(), "f64")


def test_c3_full_size():
    """The batched workload at its benchmark size (8192 FP64 segments, lengths
    floor(2^(20U)), about 6.4e8 elements generated on the device): the autotuned,
    graph-captured plan equals the direct batched call bitwise on every segment, and
    sampled segments (the longest, the shortest, random ones) meet the parity bar
    against the oracle."""
    lens = vnp_gen.log_uniform_lengths(8192, 0, 20, seed=0, stream=7)
    off = np.zeros(8193, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    total = int(off[-1])
    r = vnp_gen.recipe("c3_values")
    x = torch.empty(total, dtype=torch.float64, device="cuda")
    vnp_gen.dev_fill(x, kind=r["kind"], lo=r["lo"], hi=r["hi"], seed=r["seed"], stream=r["stream"])
    doff = torch.from_numpy(off).cuda()
    plan = vnp.Plan(x, doff, h_offsets=off, autotune=True)
    got = plan.run().clone()
    direct = vnp.nrm_batched(x, doff)
    torch.cuda.synchronize()
    print(f"c3: {total} elements, plan {plan.info()}", flush=True)
    g = got.cpu().numpy()
    assert np.array_equal(g.view(np.uint64), direct.cpu().numpy().view(np.uint64))
    order = np.argsort(lens, kind="stable")
    rng = np.random.default_rng(3)
    sample = sorted(set(order[-4:].tolist()) | set(order[:4].tolist()) | set(rng.choice(8192, 24, replace=False).tolist()))
    for s in sample:
        seg = x[int(off[s]):int(off[s + 1])].cpu().numpy()
        o = float(oracle.nrmf(seg))
        assert_parity(float(g[s]), o, seg.size, "f64", f"segment {s}, length {seg.size}")
    plan.close()
    del x


def test_indices_beyond_32_bits():
    """Element indices past 2^32 and byte offsets past 2^34.  The canonical tree's root
    over T tiles (2^k < T <= 2^(k+1)) is the node of the first 2^k tiles' root and the
    rest's root (zero padding is exact), so for binary32 and n = 2^32 + r:
    nrmf(x) = node(nrmf(x[:2^32]), nrmf(x[2^32:])) bitwise, with the node taken from a
    two-element call; one level down the same holds for x[:2^32].  Then binary64 with
    incx = +-2 over a 16 GiB buffer equals the contiguous (reversed) copy bitwise."""
    te = vnp.tile_elems(vnp.F32)
    assert te == 1 << 14
    big = 1 << 32
    n = big + 3 * te + 37
    print(f"binary32 n = {n}", flush=True)
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    vnp_gen.dev_fill(x, kind="u11", seed=11, stream=3)

    def node(a, b):
        pair = torch.stack([a, b]).contiguous()
        return vnp.nrm_batched(pair, torch.tensor([0, 2], dtype=torch.int64, device="cuda"))[0]

    whole = vnp.nrmf(x)
    left = vnp.nrmf(x[:big])
    right = vnp.nrmf(x[big:])
    assert bits(whole.item(), "f32") == bits(node(left, right).item(), "f32")
    half = big >> 1
    assert bits(left.item(), "f32") == bits(node(vnp.nrmf(x[:half]), vnp.nrmf(x[half:big])).item(), "f32")
    # a plain magnitude check: U[0, 1) elements give about sqrt(n / 3)
    assert abs(whole.item() / math.sqrt(n / 3.0) - 1.0) < 1e-3
    del x, whole, left, right
    torch.cuda.empty_cache()

    m = (1 << 30) + 5
    print(f"binary64 n = {m}, incx = +-2", flush=True)
    xd = torch.empty(2 * m, dtype=torch.float64, device="cuda")
    vnp_gen.dev_fill(xd, kind="u11", seed=12, stream=3)
    xs = xd[0:2 * m - 1:2].contiguous()
    fwd = vnp.nrmf(xd, n=m, incx=2).item()
    assert bits(fwd, "f64") == bits(vnp.nrmf(xs).item(), "f64")
    rev = vnp.nrmf(xd, n=m, incx=-2).item()
    assert bits(rev, "f64") == bits(vnp.nrmf(xs.flip(0).contiguous()).item(), "f64")
    del xd, xs
