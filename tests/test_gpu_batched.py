"""Batched norms, column norms and plans: every segment bitwise equal to the single-vector
call (same canonical tree), graph replays equal to eager calls, invalid offsets rejected."""
import math

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")


def _segments(seed, count, maxlog=18):
    L = vnp_gen.log_uniform_lengths(count, 0, maxlog, seed=seed)
    L[::7] = 0  # some empty segments
    L[1] = 1
    L[2] = 8192 * 3 + 17
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(L)
    return off


def _plain(x, off, s, p=2.0):
    seg = x[int(off[s]):int(off[s + 1])]
    if seg.numel() == 0:
        return 0.0
    r = vnp.nrmf(seg) if p == 2.0 else vnp.nrmp(seg, p)
    return r.item()


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", [2.0, 1.0, 3.0, math.inf])
def test_batched_bitwise_equals_plain(fmt, p):
    off = _segments(1, 300)
    n = int(off[-1])
    x = to_dev(vnp_gen.host_fill(n, dtype=fmt, kind="u11exp", lo=-30, hi=30, seed=2))
    res = vnp.nrm_batched(x, to_dev(off), p=p)
    torch.cuda.synchronize()
    r = res.cpu().numpy()
    print(f"batched {fmt} p={p}: {len(off) - 1} segments, {n} elements", flush=True)
    for s in range(len(off) - 1):
        assert r[s] == _plain(x, off, s, p) or (math.isnan(r[s]) and math.isnan(_plain(x, off, s, p))), s


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_batched_against_oracle(fmt):
    off = _segments(3, 64, maxlog=16)
    xh = vnp_gen.host_fill(int(off[-1]), dtype=fmt, kind="u11exp", lo=-30, hi=30, seed=4)
    r = vnp.nrm_batched(to_dev(xh), to_dev(off)).cpu().numpy()
    for s in range(len(off) - 1):
        seg = xh[off[s]:off[s + 1]]
        assert_parity(r[s], oracle.nrmf(seg, "A"), max(seg.size, 1), fmt, f"segment {s}")


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_node_via_two_element_segments(fmt):
    # segments of length 2 evaluate exactly one leaf node: compare it with cr_hypot
    dt = np.float64 if fmt == "f64" else np.float32
    rng = np.random.default_rng(5)
    k = 20000
    a = (rng.random(k) + 0.5) * np.exp2(rng.integers(-60, 60, k))
    b = a * np.exp2(-rng.random(k) * 30)
    pairs = np.stack([a, -b], axis=1).astype(dt).reshape(-1)
    off = np.arange(0, 2 * k + 1, 2, dtype=np.int64)
    r = vnp.nrm_batched(to_dev(pairs), to_dev(off)).cpu().numpy()
    eps = 2.0 ** -53 if fmt == "f64" else 2.0 ** -24
    worst = 0.0
    for i in range(k):
        x0, x1 = float(pairs[2 * i]), float(pairs[2 * i + 1])
        c = oracle.cr_hypot(x0, x1) if fmt == "f64" else oracle.cr_hypotf(x0, x1)
        worst = max(worst, abs(float(r[i]) - c) / c / eps)
    # binary64 node: relative error <= (1 + eps)^2 - 1 from the exact value, so within
    # 3 eps of the correctly rounded one; binary32 node: within 1.0001 eps (nearly correctly rounded)
    assert worst <= (3.0 if fmt == "f64" else 1.0001), worst
    z = vnp.nrm_batched(to_dev(np.stack([a.astype(dt), np.zeros(k, dt)], 1).reshape(-1)), to_dev(off)).cpu().numpy()
    assert np.array_equal(z, a.astype(dt))  # node(a, 0) = |a| exactly


def test_binary32_node_special_values_and_tiny_ratios():
    """The binary32 hypot node takes its special values from min(root, |a| + |b|): signed
    zeros give +0, an infinity gives +inf, a NaN gives NaN (also next to an infinity), and
    a smaller operand below 2^-13 of the larger leaves exactly the larger one (the
    correctly rounded result there), down to ratios of 2^-70 and into the subnormals."""
    rng = np.random.default_rng(23)
    k = 4096
    a = ((rng.random(k) + 0.5) * np.exp2(rng.integers(-100, 120, k).astype(np.float64))).astype(np.float32)
    b = (a.astype(np.float64) * np.exp2(-rng.integers(13, 71, k).astype(np.float64))
         * (rng.random(k) + 0.5)).astype(np.float32)
    sa, sb = rng.random(k) < 0.5, rng.random(k) < 0.5
    a[sa], b[sb] = -a[sa], -b[sb]
    sp = np.array([[-0.0, -0.0], [0.0, -0.0], [-0.0, 3.5], [-2.5, 0.0], [-np.inf, 1.0], [1.0, np.inf],
                   [-np.inf, -np.inf], [np.nan, 1.0], [2.0, np.nan], [-np.inf, np.nan], [np.nan, np.inf],
                   [1e-45, -1e-45], [3e38, 3e38], [-3e38, 1e-45]], dtype=np.float32)
    x = np.concatenate([np.stack([a, b], 1), sp]).reshape(-1)
    off = np.arange(0, x.size + 1, 2, dtype=np.int64)
    r = vnp.nrm_batched(to_dev(x), to_dev(off)).cpu().numpy()
    big = np.maximum(np.abs(a), np.abs(b))
    assert np.array_equal(r[:k].view(np.uint32), big.view(np.uint32))
    got = r[k:]
    assert got[0] == 0.0 and not np.signbit(got[0]) and got[1] == 0.0 and not np.signbit(got[1])
    assert got[2] == 3.5 and got[3] == 2.5
    assert np.all(np.isposinf(got[4:7]))
    assert np.all(np.isnan(got[7:11]))
    for i, (u, v) in enumerate(sp[11:]):
        c = oracle.cr_hypotf(float(u), float(v))
        g = float(got[11 + i])
        assert (g == c) if math.isinf(c) else abs(g - c) <= 2.0 ** -24 * c * 1.0001, (u, v, g, c)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("p", [2.0, 3.0, 0.5])
def test_node_symmetric_and_monotone(fmt, p):
    """node(a, b) == node(b, a) bitwise, and the node is non-decreasing in each operand:
    for fixed b, increasing |a| never lowers the value -- by one ulp for the hypot node
    (correctly rounded operations only), over a wide sweep for every node (the p node's
    polynomial evaluation is monotone only to within its error).  Pairs cover ratios
    1 .. 2^-70 and the scaled ranges (tiny, huge, zero, inf)."""
    dt = np.float64 if fmt == "f64" else np.float32
    rng = np.random.default_rng(11)
    k = 8192
    lo_e, hi_e = (-1060, 1010) if fmt == "f64" else (-140, 120)
    a = (rng.random(k) + 0.5) * np.exp2(rng.integers(lo_e, hi_e, k).astype(np.float64))
    b = a * np.exp2(-rng.random(k) * 70)
    a[:8], b[:8] = [0, 1, np.inf, 3, 0, 2.0 ** lo_e, 5, 1], [0, 0, 2, np.inf, 7, 2.0 ** lo_e, 5, 1]
    a, b = a.astype(dt), b.astype(dt)
    off = np.arange(0, 2 * k + 1, 2, dtype=np.int64)
    doff = to_dev(off)

    def node(x, y):
        return vnp.nrm_batched(to_dev(np.stack([x, y], 1).reshape(-1)), doff, p=p).cpu().numpy()

    ab, ba = node(a, -b), node(-b, a)
    assert np.array_equal(ab.view(np.uint64 if fmt == "f64" else np.uint32),
                          ba.view(np.uint64 if fmt == "f64" else np.uint32))
    if p == 2.0:  # consecutive values of the first operand
        a_up = np.nextafter(a, np.inf)
        fin = np.isfinite(a_up)
        assert np.all(node(a_up, b)[fin] >= ab[fin])
    # a sweep of the first operand at a fixed second operand
    for b0 in (1.0, 2.0 ** -30, 2.0 ** (lo_e + 20)):
        sweep = np.sort(np.exp2(rng.uniform(lo_e, hi_e, k))).astype(dt)
        r = node(sweep, np.full(k, b0, dt))
        assert np.all(np.diff(r) >= 0)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_column_norms(fmt):
    m, ncols, lda = 20000, 37, 20011
    A = vnp_gen.host_fill(lda * ncols, dtype=fmt, kind="exp", lo=-10, hi=10, seed=6)
    d = to_dev(A)
    r = vnp.nrmf_cols(d, m, ncols, lda).cpu().numpy()
    for j in range(ncols):
        assert r[j] == vnp.nrmf(d[j * lda:j * lda + m]).item()


@pytest.mark.parametrize("fmt", ["f64", "f32"])
def test_plan_graph_replays(fmt):
    off = _segments(7, 500)
    n = int(off[-1])
    x = to_dev(vnp_gen.host_fill(n, dtype=fmt, kind="u11exp", lo=-30, hi=30, seed=8))
    doff = to_dev(off)
    plan = vnp.Plan(x, doff, h_offsets=off, autotune=True)
    print("plan shape", plan.info(), flush=True)
    for rep in range(4):
        vnp_gen.dev_fill(x, kind="u11exp", lo=-30, hi=30, seed=100 + rep)
        got = plan.run().clone()
        torch.cuda.synchronize()
        ref = vnp.nrm_batched(x, doff)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
    plan.close()


def test_invalid_offsets_give_nan_without_reading():
    x = torch.ones(1000, dtype=torch.float64, device="cuda")
    off = to_dev(np.array([0, 10, 5000], dtype=np.int64))  # second segment runs past the end
    r = vnp.nrm_batched(x, off).cpu().numpy()
    assert np.all(np.isnan(r))
    ok = vnp.nrm_batched(x, to_dev(np.array([0, 10, 1000], dtype=np.int64))).cpu().numpy()
    assert ok[0] == vnp.nrmf(x[:10]).item() and ok[1] == vnp.nrmf(x[10:]).item()


def test_batched_argument_errors():
    L = vnp.lib()
    assert L.vnp_dnrmf_batched(-1, 0, 0, 0, 0, None) == -1
    assert L.vnp_dnrmf_batched(3, 0, 10, 0, 0, None) == -2
    assert L.vnp_dnrmf_cols(5, 2, 1, 4, 1, None) == -4


def test_p_plan_outlives_finalize():
    """A p-norm plan keeps its own copy of the p node's table: after vnp_finalize (which
    releases the shared tables and workspaces) its replays still equal the plain calls."""
    off = _segments(9, 120)
    n = int(off[-1])
    x = to_dev(vnp_gen.host_fill(n, dtype="f64", kind="u11exp", lo=-20, hi=20, seed=12))
    doff = to_dev(off)
    plan = vnp.Plan(x, doff, p=3.0, h_offsets=off, autotune=False)
    first = plan.run().clone()
    torch.cuda.synchronize()
    vnp.finalize()
    again = plan.run().clone()
    torch.cuda.synchronize()
    ref = vnp.nrm_batched(x, doff, p=3.0)
    torch.cuda.synchronize()
    assert torch.equal(first, ref) and torch.equal(again, ref)
    plan.close()


@pytest.mark.parametrize("fmt,p", [("f64", 2.0), ("f32", 2.0), ("f64", 3.0)])
def test_long_segment_multipass_finish(fmt, p):
    """One segment of more than 512 runs (2^25 + 7 FP64 or 2^26 + 7 FP32 elements: 4097
    tiles, above the 4096 runs a segment may have, so 2049 runs of two tiles at the default
    shape) among about a hundred short ones: its run roots are reduced by the finish kernel
    in several passes.  Bitwise equal to the plain call and within the parity bound of the
    oracle."""
    long_n = (1 << 25) + 7 if fmt == "f64" else (1 << 26) + 7
    L = vnp_gen.log_uniform_lengths(100, 0, 13, seed=21)
    L[40] = long_n
    off = np.zeros(L.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(L)
    xh = vnp_gen.host_fill(int(off[-1]), dtype=fmt, kind="u11exp", lo=-30, hi=30, seed=22)
    x = to_dev(xh)
    print(f"multi-pass finish {fmt} p={p}: {L.size} segments, long one {long_n}", flush=True)
    r = vnp.nrm_batched(x, to_dev(off), p=p).cpu().numpy()
    for s in range(L.size):
        assert r[s] == _plain(x, off, s, p), s
    for s in (40, 0, 39, 41, 99):
        seg = xh[off[s]:off[s + 1]]
        o = oracle.nrmf(seg, "A") if p == 2.0 else oracle.nrmp(seg, p)
        assert_parity(r[s], o, max(seg.size, 1), fmt, f"segment {s}")


def test_autotune_cache_file(tmp_path, monkeypatch):
    """The autotune record is written to the VNP_AUTOTUNE_CACHE file as JSON, read back by a
    later plan of the same class without timing (a shape edited into the file is the shape
    the next plan takes), replaced by autotune = 2, and never changes a result."""
    import json

    path = tmp_path / "autotune.json"
    monkeypatch.setenv("VNP_AUTOTUNE_CACHE", str(path))
    vnp.autotune_cache_clear()
    try:
        off = _segments(5, 200)
        n = int(off[-1])
        x = to_dev(vnp_gen.host_fill(n, dtype="f64", kind="u11exp", lo=-30, hi=30, seed=6))
        d_off = to_dev(off)
        p1 = vnp.Plan(x, d_off, autotune=1)
        ref = p1.run().clone()
        torch.cuda.synchronize()
        doc = json.loads(path.read_text())
        entries = doc["entries"]
        assert len(entries) == 1
        key, rec = next(iter(entries.items()))
        print("autotune record:", key, rec, p1.info(), flush=True)
        assert "f64" in key and "hypot" in key and f"tree{vnp.tree_id(vnp.F64):x}" in key
        assert p1.info()["tiles_per_item"] == 1 << rec["lwt"] and p1.info()["waves_per_block"] == rec["wpb"]
        # a different, valid shape edited into the file: the next plan of the class takes it
        edited = {"lwt": 3 if rec["lwt"] != 3 else 1, "wpb": 4 if rec["wpb"] != 4 else 8, "blocks": 256, "ms": 9.0}
        # in the writer's one-line entry form, which the reader parses
        path.write_text('{\n  "version": 1,\n  "entries": {\n    "%s": {"lwt": %d, "wpb": %d, "blocks": %d, '
                        '"ms": 9.0000}\n  }\n}\n' % (key, edited["lwt"], edited["wpb"], edited["blocks"]))
        vnp.autotune_cache_clear()
        p2 = vnp.Plan(x, d_off, autotune=1)
        info = p2.info()
        assert info["tiles_per_item"] == 1 << edited["lwt"] and info["waves_per_block"] == edited["wpb"], info
        assert info["blocks"] <= edited["blocks"]
        assert torch.equal(p2.run(), ref)
        # autotune = 2 times again and replaces the record
        p3 = vnp.Plan(x, d_off, autotune=2)
        assert torch.equal(p3.run(), ref)
        rec3 = json.loads(path.read_text())["entries"][key]
        assert rec3["ms"] != 9.0
        for p in (p1, p2, p3):
            p.close()
    finally:
        monkeypatch.delenv("VNP_AUTOTUNE_CACHE")
        vnp.autotune_cache_clear()
