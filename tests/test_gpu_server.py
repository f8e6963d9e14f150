"""Request server: each result bitwise equal to the plain call, alone and in any mix, and
within the parity bound of the oracle (A for p = 2, A_p otherwise; Sect. 2 and 4);
admission by device memory; invalid requests fail in isolation; injected batch failures
recover; destroy completes what it drops; the open-loop load generator runs end to end."""
import ctypes
import math
import threading
import time

import numpy as np
import pytest

import oracle
import vnp_gen
from gpu_util import assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
vnp = pytest.importorskip("paper_2509_06220_amd")


def plain(ptr, n, dtype, p, incx):
    dt = torch.float64 if dtype == vnp.F64 else torch.float32
    out = torch.empty((), dtype=dt, device="cuda")
    L = vnp.lib()
    s = torch.cuda.current_stream().cuda_stream
    if p == 2.0:
        fn = L.vnp_dnrmf if dtype == vnp.F64 else L.vnp_snrmf
        assert fn(n, ptr, incx, out.data_ptr(), s) == 0
    else:
        fn = L.vnp_dnrmp if dtype == vnp.F64 else L.vnp_snrmp
        assert fn(n, ptr, incx, p, out.data_ptr(), s) == 0
    return float(out.item())


def fill_request(ptr, n, dtype, incx, seed, stream):
    span = (n - 1) * abs(incx) + 1 if n > 0 else 1
    vnp_gen.dev_fill_ptr(ptr, span, "f64" if dtype == vnp.F64 else "f32", kind="u11exp", lo=-30, hi=30,
                         seed=seed, stream=stream, hip_stream=torch.cuda.current_stream().cuda_stream)


def logical_host(n, dtype, incx, seed, stream):
    """The request's logical elements (BLAS stride order) from the host generator."""
    fmt = "f64" if dtype == vnp.F64 else "f32"
    span = (n - 1) * abs(incx) + 1 if n > 0 else 1
    buf = vnp_gen.host_fill(span, dtype=fmt, kind="u11exp", lo=-30, hi=30, seed=seed, stream=stream)
    v = buf[::abs(incx)][:n]
    return np.ascontiguousarray(v[::-1] if incx < 0 else v)


def oracle_value(v, p):
    return float(oracle.nrmf(v, "A")) if p == 2.0 else float(oracle.nrmp(v, p))


def check_oracle(value, n, dtype, p, incx, seed, stream, note=""):
    v = logical_host(n, dtype, incx, seed, stream)
    assert_parity(value, oracle_value(v, p), max(n, 1), "f64" if dtype == vnp.F64 else "f32",
                  f"{note} n={n} dtype={dtype} p={p} incx={incx}")


def make_requests(srv, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        dtype = vnp.F64 if rng.random() < 0.7 else vnp.F32
        p = 2.0 if rng.random() < 0.6 else float(rng.choice([1.0, 3.0, 4.5, math.inf]))
        n = int(np.floor(2 ** rng.uniform(0, 17)))
        incx = int(rng.choice([1, 1, 1, 2, -1, -3]))
        esz = 8 if dtype == vnp.F64 else 4
        span = (n - 1) * abs(incx) + 1 if n > 0 else 1
        ptr = srv.alloc(span * esz)
        assert ptr is not None
        fill_request(ptr, n, dtype, incx, seed, i)
        reqs.append((ptr, n, dtype, p, incx))
    torch.cuda.synchronize()
    return reqs


def same(a, b):
    return a == b or (math.isnan(a) and math.isnan(b))


def blocker(srv, n=1 << 30):
    """A long FP64 p = 3 request (about 2.5 ms on the device) that keeps the server's only
    stream busy while a burst queues up behind it; returns its buffer and request."""
    buf = torch.empty(n, dtype=torch.float64, device="cuda")
    vnp_gen.dev_fill(buf, kind="u11", seed=77)
    torch.cuda.synchronize()
    return buf, vnp.Request(vnp.F64, 3.0, n, buf.data_ptr(), 1)


def burst(srv, reqs, blk=None):
    """All requests submitted back to back from native code.  With a blocker, the blocker is
    submitted first and, once it is in flight, the burst follows about 0.1 ms later (the
    load generator's arrival times are relative to 2 ms after its start), so the whole burst
    queues behind it and forms one batch."""
    tk = None
    if blk is not None:
        tk = srv.submit(blk.x, blk.n, blk.dtype, blk.p, blk.incx)
        while srv.stats()["in_flight"] == 0:  # the blocker is on the device before the burst starts
            time.sleep(0.00002)
    arr = (vnp.Request * len(reqs))(*reqs)
    lat, val, st, wall = vnp_gen.run_load(srv, np.full(len(reqs), -0.0019 if blk is not None else 0.0), arr)
    if tk is not None:
        assert srv.wait(tk).status == 0
    return val, st


def test_results_equal_alone_and_in_the_mix():
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=64, streams=3, max_wait_us=100)
    reqs = make_requests(srv, 150, seed=1)
    ref = [plain(*r) for r in reqs]
    tickets = [srv.submit(ptr, n, dtype, p, incx) for ptr, n, dtype, p, incx in reqs]  # one burst
    mixed = [srv.wait(t) for t in tickets]
    for i, (r, m) in enumerate(zip(ref, mixed)):
        assert m.status == 0 and same(m.value, r) and m.t_done_ns >= m.t_submit_ns
        _, n, dtype, p, incx = reqs[i]
        check_oracle(m.value, n, dtype, p, incx, 1, i, "in the mix")
    for i, ((ptr, n, dtype, p, incx), r) in enumerate(zip(reqs[:40], ref[:40])):  # alone
        a = srv.wait(srv.submit(ptr, n, dtype, p, incx))
        assert a.status == 0 and same(a.value, r)
        check_oracle(a.value, n, dtype, p, incx, 1, i, "alone")
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == 190 and st["batches"] >= 3 and st["max_batch_seen"] > 1
    srv.close()


def test_long_requests_alone():
    """Long requests sent one at a time (each batch of one is the single-vector call) give
    the plain call's bits."""
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=8, streams=1, max_wait_us=0)
    hs = torch.cuda.current_stream().cuda_stream
    for dtype, n, incx in ((vnp.F64, (1 << 23) + 5, 1), (vnp.F32, (1 << 24) + 3, 1), (vnp.F64, (1 << 22) + 1, 2),
                           (vnp.F64, (1 << 23) + 5, -1)):
        esz = 8 if dtype == vnp.F64 else 4
        span = (n - 1) * abs(incx) + 1
        ptr = srv.alloc(span * esz)
        vnp_gen.dev_fill_ptr(ptr, span, "f64" if dtype == vnp.F64 else "f32", kind="u11exp", lo=-30, hi=30,
                             seed=9, stream=n, hip_stream=hs)
        torch.cuda.synchronize()
        for p in (2.0, 3.0):
            print(f"long request dtype={dtype} n={n} incx={incx} p={p}", flush=True)
            r = srv.wait(srv.submit(ptr, n, dtype, p, incx))
            assert r.status == 0 and same(r.value, plain(ptr, n, dtype, p, incx))
            if p == 2.0:
                v = vnp_gen.host_fill(span, dtype="f64" if dtype == vnp.F64 else "f32", kind="u11exp", lo=-30,
                                      hi=30, seed=9, stream=n)[::abs(incx)][:n]
                assert_parity(r.value, oracle_value(np.ascontiguousarray(v[::-1] if incx < 0 else v), p), n,
                              "f64" if dtype == vnp.F64 else "f32", "long request alone")
        srv.free(ptr)
    srv.close()


def test_concurrent_clients():
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=128, streams=4, max_wait_us=0)
    reqs = make_requests(srv, 160, seed=2)
    ref = [plain(*r) for r in reqs]
    got = [None] * len(reqs)

    def client(k):
        for i in range(k, len(reqs), 4):
            ptr, n, dtype, p, incx = reqs[i]
            got[i] = srv.wait(srv.submit(ptr, n, dtype, p, incx))

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for g, r in zip(got, ref):
        assert g.status == 0 and same(g.value, r)
    srv.close()


def test_admission_by_device_memory():
    srv = vnp.Server(pool_bytes=1 << 20, max_batch=8, streams=1)
    a = srv.alloc(600_000)
    assert a is not None
    assert srv.alloc(600_000) is None  # pool full: back-pressure
    srv.free(a)
    b = srv.alloc(600_000)
    assert b is not None
    assert srv.stats()["pool_free_bytes"] < (1 << 20)
    srv.free(b)
    assert srv.stats()["pool_free_bytes"] == (1 << 20)
    with pytest.raises(vnp.VnpError):
        srv.free(b)  # not a live block
    srv.close()


def test_invalid_requests_fail_alone():
    srv = vnp.Server(pool_bytes=1 << 24, max_batch=32, streams=2, max_wait_us=200)
    ptr = srv.alloc(8 * 1000)
    vnp_gen.dev_fill_ptr(ptr, 1000, "f64", kind="u11", seed=3, hip_stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ok = plain(ptr, 1000, vnp.F64, 2.0, 1)
    t = [srv.submit(ptr, 1000, vnp.F64, 2.0, 1), srv.submit(ptr, -1, vnp.F64, 2.0, 1),
         srv.submit(ptr, 1000, vnp.F64, 2.0, 0), srv.submit(ptr, 1000, vnp.F64, -1.0, 1),
         srv.submit(None, 5, vnp.F64, 2.0, 1), srv.submit(ptr, 0, vnp.F64, 2.0, 1),
         srv.submit(ptr, 1000, vnp.F64, 2.0, 1)]
    r = [srv.wait(x) for x in t]
    assert [x.status for x in r] == [0, -3, -5, -2, -4, 0, 0]
    assert r[0].value == ok and r[6].value == ok and r[5].value == 0.0
    with pytest.raises(vnp.VnpError):
        srv.poll(t[0])
    srv.close()


def test_injected_batch_failures_are_rerun():
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=16, streams=2, max_wait_us=500, inject_failure_every=2)
    reqs = make_requests(srv, 60, seed=4)
    ref = [plain(*r) for r in reqs]
    tickets = [srv.submit(*r[:2], r[2], r[3], r[4]) for r in reqs]
    for tk, r in zip(tickets, ref):
        g = srv.wait(tk)
        assert g.status == 0 and same(g.value, r)
    assert srv.stats()["failed_batches"] >= 1
    srv.close()


def test_open_loop_load_generator():
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=256, streams=4, max_wait_us=20)
    reqs = make_requests(srv, 300, seed=5)
    ref = [plain(*r) for r in reqs]
    arr = (vnp.Request * len(reqs))(*[vnp.Request(d, p, n, ptr, inc) for ptr, n, d, p, inc in reqs])
    rng = np.random.default_rng(6)
    arrival = np.cumsum(rng.exponential(1 / 20000.0, len(reqs)))
    lat, val, st, wall = vnp_gen.run_load(srv, arrival, arr)
    assert np.all(st == 0)
    assert all(same(v, r) for v, r in zip(val, ref))
    assert np.all(lat > 0) and wall > arrival[-1]
    print(f"load: p50 {np.percentile(lat, 50) * 1e6:.0f} us, p99 {np.percentile(lat, 99) * 1e6:.0f} us", flush=True)
    srv.close()


def test_many_classes_in_one_batch():
    """A batch of more (dtype, p) classes than a descriptor buffer sized for 32 would hold:
    63 requests with distinct p, queued behind a blocker, launch as one batch."""
    srv = vnp.Server(pool_bytes=1 << 28, max_batch=63, streams=1, max_wait_us=200000)
    buf, blk = blocker(srv)
    reqs, meta = [], []
    for i in range(63):
        dtype = vnp.F64 if i % 3 else vnp.F32
        p = 1.03 + 0.11 * i  # 63 distinct p, none of 1, 2 or inf
        n, incx = 3000 + 37 * i, (1, 2, -1)[i % 3]
        esz = 8 if dtype == vnp.F64 else 4
        ptr = srv.alloc(((n - 1) * abs(incx) + 1) * esz)
        fill_request(ptr, n, dtype, incx, 11, i)
        reqs.append(vnp.Request(dtype, p, n, ptr, incx))
        meta.append((ptr, n, dtype, p, incx))
    torch.cuda.synchronize()
    val, st = burst(srv, reqs, blk)
    assert np.all(st == 0)
    stats = srv.stats()
    print("many classes:", stats, flush=True)
    assert stats["max_batch_seen"] > 32
    for i, (ptr, n, dtype, p, incx) in enumerate(meta):
        r = plain(ptr, n, dtype, p, incx)
        assert same(val[i], r), (i, val[i], r)
        check_oracle(val[i], n, dtype, p, incx, 11, i, "distinct-p batch")
    srv.close()
    del buf


def test_long_requests_in_a_mixed_batch():
    """Requests of more than 512 run roots inside a batch of several requests: their run
    roots are reduced by the multi-pass finish (one tile per work item, 2048 runs)."""
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=16, streams=1, max_wait_us=200000)
    buf, blk = blocker(srv)
    specs = [(vnp.F64, (1 << 24) + 5, 2.0, 1), (vnp.F64, (1 << 24) + 5, 3.0, -1), (vnp.F32, (1 << 25) + 3, 2.0, 1),
             (vnp.F64, 5000, 2.0, 1), (vnp.F32, 777, 3.0, 2), (vnp.F64, 100000, 2.0, -2)]
    reqs, meta = [], []
    for i, (dtype, n, p, incx) in enumerate(specs):
        esz = 8 if dtype == vnp.F64 else 4
        ptr = srv.alloc(((n - 1) * abs(incx) + 1) * esz)
        assert ptr is not None
        fill_request(ptr, n, dtype, incx, 13, i)
        reqs.append(vnp.Request(dtype, p, n, ptr, incx))
        meta.append((ptr, n, dtype, p, incx))
    torch.cuda.synchronize()
    val, st = burst(srv, reqs, blk)
    assert np.all(st == 0)
    stats = srv.stats()
    print("mixed long batch:", stats, flush=True)
    assert stats["max_batch_seen"] == len(specs)  # the burst formed one batch behind the blocker
    for i, (ptr, n, dtype, p, incx) in enumerate(meta):
        print(f"  request {i}: n={n} dtype={dtype} p={p} incx={incx}", flush=True)
        assert same(val[i], plain(ptr, n, dtype, p, incx)), i
        check_oracle(val[i], n, dtype, p, incx, 13, i, "mixed long batch")
    srv.close()
    del buf


def test_p_outside_the_working_precision_is_rejected():
    """p whose reciprocal overflows the request's dtype is invalid (-2), alone and in a
    burst; the valid requests of the same burst are unaffected."""
    srv = vnp.Server(pool_bytes=1 << 24, max_batch=16, streams=2, max_wait_us=100)
    ptr = srv.alloc(8 * 4000)
    fill_request(ptr, 4000, vnp.F64, 1, 5, 0)
    torch.cuda.synchronize()
    good = plain(ptr, 4000, vnp.F64, 3.0, 1)
    reqs = [vnp.Request(vnp.F64, 1e-310, 4000, ptr, 1), vnp.Request(vnp.F32, 1e-39, 4000, ptr, 1),
            vnp.Request(vnp.F32, 1e-50, 4000, ptr, 1), vnp.Request(vnp.F64, 3.0, 4000, ptr, 1),
            vnp.Request(vnp.F64, 0.0, 4000, ptr, 1), vnp.Request(vnp.F64, 3.0, 4000, ptr, 1)]
    val, st = burst(srv, reqs)
    assert list(st) == [-2, -2, -2, 0, -2, 0]
    assert val[3] == good and val[5] == good
    srv.close()


def test_destroy_completes_dropped_requests():
    """Requests still queued when the server is destroyed complete as VNP_ECANCELED, and a
    client blocked in wait returns before the server is freed."""
    srv = vnp.Server(pool_bytes=1 << 24, max_batch=1, streams=1, max_wait_us=0)
    buf, blk = blocker(srv)
    ptr = srv.alloc(8 * 1000)
    fill_request(ptr, 1000, vnp.F64, 1, 6, 0)
    torch.cuda.synchronize()
    ok = plain(ptr, 1000, vnp.F64, 2.0, 1)
    # 40 blockers run one after another (max_batch 1, one stream): tens of milliseconds
    tickets = [srv.submit(blk.x, blk.n, vnp.F64, 3.0, 1) for _ in range(40)]
    tickets += [srv.submit(ptr, 1000) for _ in range(30)]
    got = {}
    h = srv.handle

    def waiter():
        r = vnp.Result()
        got["rc"] = vnp.lib().vnp_server_wait(h, tickets[-1], -1, ctypes.byref(r))
        got["last"] = r

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.005)  # the waiter blocks inside vnp_server_wait (ctypes releases the GIL)
    srv.close()
    th.join(timeout=60)
    assert not th.is_alive()
    assert got["rc"] == 0
    last = got["last"]
    assert (last.status == 0 and last.value == ok) or (last.status == vnp.ECANCELED and math.isnan(last.value))
    del buf


def test_admission_by_copy_matches_the_plain_call_and_the_oracle():
    """Payloads outside the pool (caller tensors, strided and reversed too) are copied into
    pool blocks at admission; a pool smaller than one burst's payloads makes later copies
    wait for memory (counted), and every result equals the plain call on the caller's data
    and stays within the oracle's parity bound.  A payload larger than the whole pool
    completes with VNP_ENOMEM; blocks are all returned at the end."""
    pool = 4 << 20
    srv = vnp.Server(pool_bytes=pool, max_batch=32, streams=2, max_wait_us=50)
    rng = np.random.default_rng(41)
    bufs, reqs, meta = [], [], []
    for i in range(120):
        dtype = vnp.F64 if rng.random() < 0.7 else vnp.F32
        p = 2.0 if rng.random() < 0.7 else float(rng.choice([1.0, 3.0, 4.5]))
        n = int(np.floor(2 ** rng.uniform(4, 18.5)))  # up to 370k elements: 3 MB FP64
        incx = int(rng.choice([1, 1, 1, 2, -1]))
        span = (n - 1) * abs(incx) + 1
        t = torch.empty(span, dtype=torch.float64 if dtype == vnp.F64 else torch.float32, device="cuda")
        fill_request(t.data_ptr(), n, dtype, incx, 21, i)
        bufs.append(t)
        reqs.append(vnp.Request(dtype, p, n, t.data_ptr(), incx))
        meta.append((t.data_ptr(), n, dtype, p, incx))
    big = torch.zeros(pool // 8 + 100, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    arr = (vnp.Request * len(reqs))(*reqs)
    lat, val, st, wall = vnp_gen.run_load(srv, np.zeros(len(reqs)), arr, copy=True)
    assert np.all(st == 0), st
    stats = srv.stats()
    print("admission by copy:", stats, flush=True)
    assert stats["admission_waits"] > 0 and stats["pool_free_bytes"] == pool
    for i, (ptr, n, dtype, p, incx) in enumerate(meta):
        assert same(val[i], plain(ptr, n, dtype, p, incx)), i
        if i % 4 == 0:
            check_oracle(val[i], n, dtype, p, incx, 21, i, "admitted by copy")
    r = srv.wait(srv.submit(big.data_ptr(), big.numel(), vnp.F64, 2.0, 1, copy=True))
    assert r.status == vnp.ENOMEM and math.isnan(r.value)
    srv.close()
