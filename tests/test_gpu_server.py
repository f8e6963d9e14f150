"""Request server: each result bitwise equal to the plain call, alone and in any mix;
admission by device memory; invalid requests fail in isolation; injected batch failures
recover; the open-loop load generator runs end to end."""
import math
import threading

import numpy as np
import pytest

import vnp_gen

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
        vnp_gen.dev_fill_ptr(ptr, span, "f64" if dtype == vnp.F64 else "f32", kind="u11exp", lo=-30, hi=30,
                             seed=seed, stream=i, hip_stream=torch.cuda.current_stream().cuda_stream)
        reqs.append((ptr, n, dtype, p, incx))
    torch.cuda.synchronize()
    return reqs


def same(a, b):
    return a == b or (math.isnan(a) and math.isnan(b))


def test_results_equal_alone_and_in_the_mix():
    srv = vnp.Server(pool_bytes=1 << 30, max_batch=64, streams=3, max_wait_us=100)
    reqs = make_requests(srv, 150, seed=1)
    ref = [plain(*r) for r in reqs]
    tickets = [srv.submit(ptr, n, dtype, p, incx) for ptr, n, dtype, p, incx in reqs]  # one burst
    mixed = [srv.wait(t) for t in tickets]
    for r, m in zip(ref, mixed):
        assert m.status == 0 and same(m.value, r) and m.t_done_ns >= m.t_submit_ns
    for (ptr, n, dtype, p, incx), r in zip(reqs[:40], ref[:40]):  # alone
        a = srv.wait(srv.submit(ptr, n, dtype, p, incx))
        assert a.status == 0 and same(a.value, r)
    st = srv.stats()
    print("server stats", st, flush=True)
    assert st["completed"] == 190 and st["batches"] >= 3 and st["max_batch_seen"] > 1
    srv.close()


def test_long_requests_alone():
    """Single long requests (one tile per work item, more than 512 run roots per request,
    reduced in several passes) give the plain call's bits."""
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
