"""Benchmark: DNRMF GB/s and fraction of the HBM roofline at n = 2^30 (FP64), plus the
batched and served modes, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]

One step = one DNRMF call (one kernel launch) over the device-resident synthetic vector
x_i = +-u_i 2^e_i, u_i in [1/2, 1), e_i in [-20, 20] (seed 0), n = 2^30.  The K timed
steps are bracketed by torch.cuda.synchronize(); each launch is also bracketed by HIP
events on the stream it runs on, giving the kernel's average duration for the roofline.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DNRMF GB/s & % HBM peak at n=2^30; batched norms/s vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dnrmf_c1.json")
KERNEL_SOURCES = ["paper_2509_06220_amd/csrc/vnp_nrm.hip", "paper_2509_06220_amd/csrc/vnp_tree.hpp",
                  "paper_2509_06220_amd/csrc/vnp_node.hpp", "paper_2509_06220_amd/csrc/vnp_internal.hpp"]


PNODE_SOURCES = ["paper_2509_06220_amd/csrc/vnp_nrm.hip", "paper_2509_06220_amd/csrc/vnp_tree.hpp",
                 "paper_2509_06220_amd/csrc/vnp_nodes_p.hpp", "paper_2509_06220_amd/csrc/vnp_internal.hpp"]
VALU_FILE = os.path.join(ROOT, "profiles", "valu_fp64.json")
FP64_PEAK_TFLOPS = 78.6
# VALU issue rate: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD every 4 clocks
# (16 lanes per clock; binary64 FMA, MUL, ADD and 32-bit integer operations alike)
VALU_PEAK_TLANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12


def pnode_hash() -> str:
    h = hashlib.sha256()
    for p in PNODE_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pnode_counters():
    """Counter summary of the DNRMP (p = 3, n = 2^28) launch (FP64 FLOPs, VALU instructions
    per node, VALUBusy) from the committed profile, if it matches the kernel sources."""
    try:
        with open(VALU_FILE) as f:
            v = json.load(f)
    except (OSError, ValueError):
        return {}
    if v.get("kernel_sha_p") != pnode_hash():
        return {}
    return v.get("dnrmp_3", {})


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per launch from the committed counter summary, if it matches the kernel."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def time_steps(fn, steps, warmup, stream, min_warm_s=0.5):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_warm_s:  # let clocks settle (untimed)
        fn()
        torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    return wall, per


def cpu_baseline(n_sample: int):
    import numpy as np

    import oracle
    import vnp_gen

    x = vnp_gen.host_fill(n_sample, kind="exp", lo=-20, hi=20, seed=0)
    threads = oracle.default_threads()
    oracle.nrmf(x[:4096], "A", threads=threads)
    t0 = time.perf_counter()
    oracle.nrmf(x, "A", threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(n_sample * 8 / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"first 2^{int(np.log2(n_sample))} elements of the n=2^30 vector, "
                      f"O-A (R with correctly rounded hypot), {threads} threads, {dt:.2f} s"}, x


def oracle_timings(x_c1):
    """The oracle's recursions A and H timed on the host, single-threaded and on all the
    threads it uses: C0 (n = 2^20, U[-1,1), seed 0) with both, and the C1 vector (x_c1,
    2^30 elements) with H (A on all threads is the CPU baseline); with the CPU model and
    core count (informational)."""
    import os

    import oracle
    import vnp_gen

    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = oracle.default_threads()
    r0 = vnp_gen.recipe("c0")
    x0 = vnp_gen.host_fill(r0["n"], kind=r0["kind"], seed=r0["seed"], stream=r0["stream"])
    out = {"cpu_model": model, "nproc": os.cpu_count(), "threads": threads, "runs": {}}

    def run(tag, x, method, th):
        oracle.nrmf(x[:4096], method, threads=th)
        t0 = time.perf_counter()
        oracle.nrmf(x, method, threads=th)
        dt = time.perf_counter() - t0
        out["runs"][tag] = {"s": round(dt, 4), "GB/s": round(x.size * 8 / dt / 1e9, 4)}

    for method in ("A", "H"):
        run(f"C0 O-{method} 1 thread", x0, method, 1)
        run(f"C0 O-{method} {threads} threads", x0, method, threads)
    run(f"C1 O-H 1 thread", x_c1, "H", 1)
    run(f"C1 O-H {threads} threads", x_c1, "H", threads)
    return out


def extra_modes(torch, vnp, vnp_gen):
    """Throughput of the other paths (informational; the headline is DNRMF)."""
    out = {}
    try:
        # small case: n = 2^20, x = U[-1,1) (seed 0); latency of one call (kernel time by HIP
        # events), cache-resident and after 512 MB of writes have evicted it
        r0 = vnp_gen.recipe("c0")
        s = torch.cuda.current_stream()
        flush = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
        for dt, key in ((torch.float64, "c0_dnrmf"), (torch.float32, "c0_snrmf")):
            x0 = torch.empty(r0["n"], dtype=dt, device="cuda")
            vnp_gen.dev_fill(x0, kind=r0["kind"], seed=r0["seed"], stream=r0["stream"])
            r = torch.empty((), dtype=dt, device="cuda")
            _, per = time_steps(lambda: vnp.nrmf(x0, out=r), 50, 10, s, min_warm_s=0.2)
            warm = statistics.median(per)
            cold = []
            for _ in range(20):
                flush.fill_(1.0)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(s)
                vnp.nrmf(x0, out=r)
                b.record(s)
                torch.cuda.synchronize()
                cold.append(a.elapsed_time(b))
            nb = r0["n"] * x0.element_size()
            out[key] = {"us_cache_resident": round(warm * 1e3, 2), "gbs_cache_resident": round(nb / warm / 1e6, 1),
                        "us_cache_flushed": round(statistics.median(cold) * 1e3, 2),
                        "gbs_cache_flushed": round(nb / statistics.median(cold) / 1e6, 1)}
            del x0
        del flush
        n = 1 << 30
        xs = torch.empty(n, dtype=torch.float32, device="cuda")
        vnp_gen.dev_fill(xs, kind="exp", lo=-20, hi=20, seed=0)
        res = torch.empty((), dtype=torch.float32, device="cuda")
        _, per = time_steps(lambda: vnp.nrmf(xs, out=res), 10, 2, s)
        out["snrmf_gbs"] = round(n * 4 / (statistics.mean(per) / 1e3) / 1e9, 1)
        del xs
        n = 1 << 28
        xp = torch.empty(n, dtype=torch.float64, device="cuda")
        vnp_gen.dev_fill(xp, kind="exp", lo=-10, hi=10, seed=0)
        resp = torch.empty((), dtype=torch.float64, device="cuda")
        for p in (1.0, 1.5, 3.0, 4.5, 8.0):
            _, per = time_steps(lambda: vnp.nrmp(xp, p, out=resp), 5, 1, s)
            out[f"dnrmp_p{p:g}_gbs"] = round(n * 8 / (statistics.mean(per) / 1e3) / 1e9, 1)
            if p == 3.0:
                # C2's roofline is HBM: the method moves n * 8 bytes.  The generic-p node is
                # bound by VALU issue in fact; the issue fraction and the FP64 FLOP rate below
                # count this implementation's instructions (they move when the code changes),
                # not the method's work
                pc = pnode_counters()
                t_s = statistics.mean(per) / 1e3
                gbs = n * 8 / t_s / 1e9
                fl, ipn = pc.get("flops_per_launch"), pc.get("valu_instr_per_node")
                out["dnrmp_p3_roofline"] = {
                    "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS, "achieved": round(gbs, 1),
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": n * 8,
                    "valu_instr_per_node": None if ipn is None else round(ipn, 1),
                    "valu_issue_frac": None if ipn is None else round(ipn * (n - 1) / t_s / 1e12 / VALU_PEAK_TLANE_OPS, 4),
                    "valu_busy_pct": None if not pc else round(pc.get("valu_busy_pct", 0.0), 1)}
                out["dnrmp_p3_fp64_flops_implementation_counted"] = {
                    "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS, "flops_per_launch": fl,
                    "achieved": None if fl is None else round(fl / t_s / 1e12, 2),
                    "frac": None if fl is None else round(fl / t_s / 1e12 / FP64_PEAK_TFLOPS, 4)}
        del xp
        torch.cuda.empty_cache()
        # norm of a 2^15 x 2^15 FP64 array stored with leading dimension 2^15 + 64 (column
        # norms, then the tree over columns)
        m = ncols = 1 << 15
        lda = m + 64
        A = torch.empty(lda * ncols, dtype=torch.float64, device="cuda")
        vnp_gen.dev_fill(A, kind="exp", lo=-20, hi=20, seed=0)
        _, per = time_steps(lambda: vnp.nrm_mat(A, m, ncols, lda, out=resp), 10, 2, s)
        out["dnrmf_mat_2p15x2p15_gbs"] = round(m * ncols * 8 / (statistics.mean(per) / 1e3) / 1e9, 1)
        del A
        # Schatten 1-norm (nuclear norm) of a 1024 x 1024 FP64 matrix: the singular values
        # (rocSOLVER) dominate the time
        G = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
        vnp_gen.dev_fill(G, kind="u11", seed=3)
        _, per = time_steps(lambda: vnp.schatten(G, 1024, 1024, 1024, 1.0, out=resp), 3, 1, s, min_warm_s=0.0)
        out["dschatten_p1_1024x1024_ms"] = round(statistics.mean(per), 3)
        del G
    except Exception as e:  # noqa: BLE001 -- report, do not hide the headline
        out["error"] = repr(e)
    return out


def batched_mode(torch, vnp, vnp_gen, reps=20):
    """8192 FP64 segments, lengths floor(2^(20U)), values U[-1,1) 2^e, e in [-30, 30] per
    element: one replay of the autotuned, graph-captured plan against 8192 plain calls
    issued back to back from native code on the same stream; every segment bitwise equal."""
    import numpy as np

    nseg = 8192
    lens = vnp_gen.log_uniform_lengths(nseg, 0, 20, seed=0, stream=7)
    off = np.zeros(nseg + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    total = int(off[-1])
    rv = vnp_gen.recipe("c3_values")
    x = torch.empty(total, dtype=torch.float64, device="cuda")
    vnp_gen.dev_fill(x, kind=rv["kind"], lo=rv["lo"], hi=rv["hi"], seed=rv["seed"], stream=rv["stream"])
    d_off = torch.from_numpy(off).to("cuda")
    out_b = torch.empty(nseg, dtype=torch.float64, device="cuda")
    out_l = torch.empty(nseg, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    plan = vnp.Plan(x, d_off, out=out_b, h_offsets=off, autotune=True)
    loop = lambda: vnp_gen.loop_plain("vnp_dnrmf", off, x.data_ptr(), 8, out_l.data_ptr(), 8,  # noqa: E731
                                      s.cuda_stream)
    # replays back to back between one pair of events (an event pair around every graph
    # replay adds tens of microseconds per replay)
    for _ in range(2):
        plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:  # let clocks settle (untimed)
        plan.run()
        torch.cuda.synchronize()
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev_a.record(s)
    for _ in range(reps):
        plan.run()
    ev_b.record(s)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    ev_ms = ev_a.elapsed_time(ev_b) / reps
    # the direct call (no plan: default shape, segments in their own order), timed the same way
    out_d = torch.empty(nseg, dtype=torch.float64, device="cuda")
    for _ in range(3):
        vnp.nrm_batched(x, d_off, out=out_d)
    torch.cuda.synchronize()
    ev_a.record(s)
    for _ in range(reps):
        vnp.nrm_batched(x, d_off, out=out_d)
    ev_b.record(s)
    torch.cuda.synchronize()
    direct_ms = ev_a.elapsed_time(ev_b) / reps
    same_d = int(torch.sum(out_b.view(torch.int64) == out_d.view(torch.int64)).item())
    wall_l, per_l = time_steps(loop, max(reps // 2, 2), 1, s, min_warm_s=0.3)
    torch.cuda.synchronize()
    same = int(torch.sum(out_b.view(torch.int64) == out_l.view(torch.int64)).item())
    tb = wall_b / reps
    tl = wall_l / max(reps // 2, 2)
    info = plan.info()
    plan.close()
    return {"workload": "8192 FP64 segments, L=floor(2^(20U)), x=U[-1,1)*2^e, e in [-30,30], seed 0",
            "elements": total, "bytes": total * 8,
            "batched_norms_per_s": round(nseg / tb, 1), "batched_ms": round(tb * 1e3, 4),
            "batched_event_ms_per_replay": round(ev_ms, 4),
            "batched_hbm_frac": round(total * 8 / (ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "direct_call_ms": round(direct_ms, 4),
            "direct_call_hbm_frac": round(total * 8 / (direct_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "direct_call_bitwise_equal_to_plan": same_d,
            "batched_replays_timed": reps,
            "batched_gbs": round(total * 8 / tb / 1e9, 1),
            "plain_loop_norms_per_s": round(nseg / tl, 1), "plain_loop_ms": round(tl * 1e3, 4),
            "speedup": round(tl / tb, 2), "bitwise_equal_segments": same, "segments": nseg, "plan": info}


SERVE_POOL_BYTES = 256 << 20


def served_mode(torch, vnp, vnp_gen, rates, seconds, compare_seconds, n_payloads=4096, check=64):
    """Open-loop Poisson arrivals against the request server.  Requests: L=floor(2^(4+20U)),
    FP64 with probability 0.7 else FP32, p=2 with probability 0.8 else one of {1, 3, 4.5},
    values U[-1,1) 2^e, e in [-30, 30].  Each request names one of n_payloads client buffers
    (device memory outside the server, generated on the device) and is admitted by copy at
    arrival: the server copies it into a block of its SERVE_POOL_BYTES pool (far smaller than
    the payloads), computes, and frees the block at completion; requests that find the pool
    full wait (back-pressure, counted).  Comparator: the same schedule (its first
    compare_seconds) through a server that runs one plain call per request, in arrival
    order, on one stream (max_batch 1, streams 1), with the same admission."""
    import numpy as np

    rng = np.random.default_rng(0)
    L = vnp_gen.log_uniform_lengths(n_payloads, 4, 24, seed=0, stream=11)
    is_d = rng.random(n_payloads) < 0.7
    pv = np.where(rng.random(n_payloads) < 0.8, 2.0, rng.choice([1.0, 3.0, 4.5], n_payloads))
    esz = np.where(is_d, 8, 4)
    nbytes = ((L * esz + 255) // 256) * 256
    off = np.concatenate([[0], np.cumsum(nbytes)])
    src = torch.empty(int(off[-1]) // 4, dtype=torch.float32, device="cuda")  # the client buffers
    hs = torch.cuda.current_stream().cuda_stream
    ptrs = np.zeros(n_payloads, dtype=np.uint64)
    for i in range(n_payloads):
        ptrs[i] = src.data_ptr() + int(off[i])
        vnp_gen.dev_fill_ptr(int(ptrs[i]), int(L[i]), "f64" if is_d[i] else "f32", kind="u11exp", lo=-30, hi=30,
                             seed=0, stream=100 + i, hip_stream=hs)
    torch.cuda.synchronize()
    out = {"workload": "Poisson arrivals, L=floor(2^(4+20U)), 70% FP64/30% FP32, p=2 80% else {1,3,4.5}, "
                       "x=U[-1,1)*2^e, e in [-30,30]; each request admitted by copy into the server's pool",
           "seconds_per_rate": seconds, "client_payloads": n_payloads, "client_payload_bytes": int(off[-1]),
           "pool_bytes": SERVE_POOL_BYTES, "comparator": "one plain call per request, FIFO, one stream "
           "(server with max_batch 1, streams 1, same admission)", "comparator_seconds": compare_seconds,
           "rates": {}}

    def schedule(rate, dur, seed):
        r = np.random.default_rng(seed)
        nreq = int(rate * dur * 1.2) + 16
        arr = np.cumsum(r.exponential(1.0 / rate, nreq))
        arr = arr[arr < dur]
        pick = r.integers(0, n_payloads, len(arr))
        req = vnp_gen.request_array(len(arr))
        req["dtype"] = np.where(is_d[pick], vnp.F64, vnp.F32)
        req["p"] = pv[pick]
        req["n"] = L[pick]
        req["x"] = ptrs[pick]
        req["incx"] = 1
        return arr, req, pick

    def run(srv, arr, req, pick):
        s0 = srv.stats()
        lat, val, st, wall = vnp_gen.run_load(srv, arr, req, copy=True)
        s1 = srv.stats()
        ok = st == 0
        nb = s1["batches"] - s0["batches"]
        return val, {
            "requests": int(len(arr)), "completed": int(ok.sum()), "errors": int((~ok).sum()),
            "p50_us": round(float(np.percentile(lat[ok], 50)) * 1e6, 1),
            "p99_us": round(float(np.percentile(lat[ok], 99)) * 1e6, 1),
            "norms_per_s": round(float(ok.sum()) / wall, 1),
            "gbs": round(float(np.sum((L * esz)[pick][ok])) / wall / 1e9, 2),
            "batches": int(nb), "mean_batch": round(float(len(arr)) / max(nb, 1), 2),
            "host_launch_us_per_batch": round((s1["host_launch_ns"] - s0["host_launch_ns"]) / max(nb, 1) / 1e3, 1),
            "batch_us_mean": round((s1["batch_ns"] - s0["batch_ns"]) / max(nb, 1) / 1e3, 1),
            "backpressure": int(s1["admission_waits"] - s0["admission_waits"]),
            "backpressure_wait_us_mean": round((s1["admission_wait_ns"] - s0["admission_wait_ns"]) /
                                               max(s1["admission_waits"] - s0["admission_waits"], 1) / 1e3, 1)}

    srv = vnp.Server(pool_bytes=SERVE_POOL_BYTES, max_batch=512, streams=4, max_wait_us=20)
    cmp_srv = vnp.Server(pool_bytes=SERVE_POOL_BYTES, max_batch=1, streams=1, max_wait_us=0)
    for sv in (srv, cmp_srv):  # warm-up: kernels loaded, workspaces allocated
        arr, req, _ = schedule(5000, 0.3, 99)
        vnp_gen.run_load(sv, arr, req, copy=True)
    for k, rate in enumerate(rates):
        arr, req, pick = schedule(rate, seconds, k)
        val, res = run(srv, arr, req, pick)
        # a sample re-run alone through the plain call on the client buffer: bitwise equal
        idx = np.linspace(0, len(arr) - 1, min(check, len(arr))).astype(np.int64)
        eq = 0
        for i in idx:
            j = int(pick[i])
            dt = torch.float64 if is_d[j] else torch.float32
            r = torch.empty((), dtype=dt, device="cuda")
            fn = ("vnp_dnrm" if is_d[j] else "vnp_snrm") + ("f" if pv[j] == 2.0 else "p")
            args = [int(L[j]), int(ptrs[j]), 1] + ([] if pv[j] == 2.0 else [float(pv[j])]) + [r.data_ptr(), hs]
            if getattr(vnp.lib(), fn)(*args) != 0:
                continue
            eq += int(r.item() == val[i] or (math.isnan(r.item()) and math.isnan(val[i])))
        res["sample_bitwise_equal"] = f"{eq}/{len(idx)}"
        # the comparator on the first compare_seconds of the same schedule, and the served
        # mode on the same prefix
        m = int(np.searchsorted(arr, compare_seconds))
        _, same_window = run(srv, arr[:m], req[:m], pick[:m])
        _, serial = run(cmp_srv, arr[:m], req[:m], pick[:m])
        res["same_window"] = {k2: same_window[k2] for k2 in ("requests", "p50_us", "p99_us", "norms_per_s")}
        res["comparator_plain_fifo"] = {k2: serial[k2] for k2 in ("requests", "p50_us", "p99_us", "norms_per_s",
                                                                  "backpressure")}
        out["rates"][str(rate)] = res
        print(json.dumps({"served_rate": rate, **res}), file=sys.stderr, flush=True)
    srv.close()
    cmp_srv.close()
    del src
    return out


# The synthetic accuracy study (the tester of Sect. 2 and Fig. 1 on stand-in inputs, and
# Sect. 5's Table 4 for p != 2): inputs by (distribution, format, seed); the GPU results
# are taken here and stored, and tests/accuracy_study.py runs the oracle algorithms and the
# exact references against them on any host.
STUDY_PS = {"1/2": 0.5, "2/3": 2.0 / 3.0, "1": 1.0, "sqrt2": math.sqrt(2.0), "e": math.e, "pi": math.pi}
STUDY_BINS = [0.0, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0, 4.0, 8.0, math.inf]


def study_input(vnp_gen, dist, fmt, seed, n):
    """U(0,1): the counter-based generator (seed, stream 51); N(0,1): numpy's PCG64
    standard normal (seed), rounded to the format."""
    import numpy as np

    if dist == "U(0,1)":
        return vnp_gen.host_fill(n, dtype=fmt, kind="u01", seed=seed, stream=51)
    return np.random.default_rng(seed).standard_normal(n).astype(np.float64 if fmt == "f64" else np.float32)


def accuracy_gpu_values(torch, vnp, vnp_gen, n_log2, seeds, pn_log2, pseeds, out_path):
    """The GPU results of the study, as exact hex strings, written to out_path."""
    n = 1 << n_log2
    res = {"n": n, "seeds": seeds, "frobenius": {}, "pnorm_n": 1 << pn_log2, "pnorm_seeds": pseeds, "pnorm": {}}
    for dist in ("U(0,1)", "N(0,1)"):
        for fmt in ("f64", "f32"):
            vals = []
            for sd in range(seeds):
                x = study_input(vnp_gen, dist, fmt, sd, n)
                vals.append(float(vnp.nrmf(torch.from_numpy(x).cuda()).item()).hex())
                del x
                print(f"accuracy study (GPU): {dist} {fmt} seed {sd}", file=sys.stderr, flush=True)
            res["frobenius"][f"{dist} {fmt}"] = vals
    for name, p in STUDY_PS.items():
        vals = []
        for sd in range(pseeds):
            xd = torch.empty(1 << pn_log2, dtype=torch.float64, device="cuda")
            vnp_gen.dev_fill(xd, kind="u01", seed=sd, stream=61)
            vals.append(float(vnp.nrmp(xd, p).item()).hex())
            del xd
        res["pnorm"][name] = vals
        print(f"accuracy study (GPU): p = {name}", file=sys.stderr, flush=True)
    with open(out_path, "w") as f:
        json.dump(res, f)
    return {"written": out_path}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=30)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rates", default="5000,20000,80000")
    ap.add_argument("--compare-seconds", type=float, default=2.0,
                    help="length of the schedule prefix run through the plain-call comparator")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy 5 times (scale of the HBM byte counters)")
    ap.add_argument("--accuracy-gpu", metavar="OUT_JSON", default=None,
                    help="only take the GPU results of the synthetic accuracy study and write them to OUT_JSON")
    ap.add_argument("--study-n-log2", type=int, default=29)
    ap.add_argument("--study-seeds", type=int, default=31)
    ap.add_argument("--study-pn-log2", type=int, default=26, help="n of the GPU p-norms of the study")
    ap.add_argument("--study-pseeds", type=int, default=8)
    ap.add_argument("--profile-op", default=None,
                    help="only run one operation K times for a profiler: dnrmf, snrmf (n=2^30), dnrmp:<p> "
                         "(n=2^28) or batched:<p> (the 8192 FP64 segments, direct batched call)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (sharding over several "
              "GPUs is designed but not built: aligned tile-subtree shards and one all-gather of the roots)",
              file=sys.stderr)
        sys.exit(2)

    import vnp_gen


    import torch

    import paper_2509_06220_amd as vnp

    if args.copy_calibration:
        nb = 1 << 31
        src = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        vnp_gen.dev_fill(src, kind="u11")
        for _ in range(5):
            vnp_gen.dev_copy(dst.data_ptr(), src.data_ptr(), nb, 0, torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb, "launches": 5}), flush=True)
        return

    if args.accuracy_gpu:
        r = accuracy_gpu_values(torch, vnp, vnp_gen, args.study_n_log2, args.study_seeds, args.study_pn_log2,
                                args.study_pseeds, args.accuracy_gpu)
        print(json.dumps(r), flush=True)
        return

    if args.profile_op:
        op = args.profile_op
        if op in ("dnrmf", "snrmf"):
            n, dt = 1 << 30, (torch.float64 if op == "dnrmf" else torch.float32)
            xo = torch.empty(n, dtype=dt, device="cuda")
            vnp_gen.dev_fill(xo, kind="exp", lo=-20, hi=20, seed=0)
            fn = lambda: vnp.nrmf(xo)  # noqa: E731
        elif op.startswith("dnrmp:"):
            n, pv = 1 << 28, float(op.split(":", 1)[1])
            xo = torch.empty(n, dtype=torch.float64, device="cuda")
            vnp_gen.dev_fill(xo, kind="exp", lo=-10, hi=10, seed=0)
            fn = lambda: vnp.nrmp(xo, pv)  # noqa: E731
        elif op.startswith("batched:"):
            # the C3 segments (8192 FP64 lengths floor(2^(20U)), values as in C3) through the
            # direct batched call at exponent p
            import numpy as np

            pv = float(op.split(":", 1)[1])
            lens = vnp_gen.log_uniform_lengths(8192, 0, 20, seed=0, stream=7)
            off = np.zeros(8193, dtype=np.int64)
            off[1:] = np.cumsum(lens)
            n = int(off[-1])
            rv = vnp_gen.recipe("c3_values")
            xo = torch.empty(n, dtype=torch.float64, device="cuda")
            vnp_gen.dev_fill(xo, kind=rv["kind"], lo=rv["lo"], hi=rv["hi"], seed=rv["seed"], stream=rv["stream"])
            d_off = torch.from_numpy(off).to("cuda")
            res_b = torch.empty(8192, dtype=torch.float64, device="cuda")
            fn = lambda: vnp.nrm_batched(xo, d_off, p=pv, out=res_b)  # noqa: E731
        else:
            print(f"unknown --profile-op {op}", file=sys.stderr)
            sys.exit(2)
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 0.5:  # let clocks settle (untimed)
            fn()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"profile_op": op, "n": n, "launches": args.steps, "ms_per_call": round(dt_s * 1e3, 4),
                          "gbs": round(n * xo.element_size() / dt_s / 1e9, 1)}), flush=True)
        return

    n = 1 << 30
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    vnp_gen.dev_fill(x, kind="exp", lo=-20, hi=20, seed=0)
    res = torch.empty((), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    wall, per = time_steps(lambda: vnp.nrmf(x, out=res), args.steps, args.warmup, stream)
    ms_step = wall / args.steps * 1e3
    nbytes = n * 8
    value = nbytes / (wall / args.steps) / 1e9
    kern_ms = statistics.mean(per)
    achieved = nbytes / (kern_ms / 1e3) / 1e9
    tr = traffic_per_launch()
    # empirical ceiling: a plain streaming read of the same buffer
    ceil_out = torch.empty(16384, dtype=torch.int32, device="cuda")
    _, per_read = time_steps(lambda: vnp_gen.dev_read(x.data_ptr(), nbytes, ceil_out.data_ptr(), 16384,
                                                      stream.cuda_stream), 10, 2, stream)
    read_gbs = nbytes / (statistics.mean(per_read) / 1e3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (device-generated, seeded)",
        "config": {"workload": "DNRMF, one vector, n=2^30 FP64, x=+-u*2^e, u in [1/2,1), e in [-20,20], seed 0",
                   "n": n, "incx": 1, "tree_id": hex(vnp.tree_id(0))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                     "kernel_ms_mean": round(kern_ms, 4), "kernel_ms_median": round(statistics.median(per), 4),
                     "kernel_ms_min": round(min(per), 4), "kernel_ms_max": round(max(per), 4),
                     "kernel_launches_timed": len(per),
                     "algorithmic_bytes": nbytes, "plain_read_gbs": round(read_gbs, 1)},
        "result": res.item(),
    }
    del x
    torch.cuda.empty_cache()
    if not args.no_extra:
        line["extra"] = extra_modes(torch, vnp, vnp_gen)
        torch.cuda.empty_cache()
    if not args.no_batched:
        try:
            line["batched"] = batched_mode(torch, vnp, vnp_gen)
        except Exception as e:  # noqa: BLE001 -- report, do not hide the headline
            line["batched"] = {"error": repr(e)}
        torch.cuda.empty_cache()
    if not args.no_serve:
        try:
            rates = [int(r) for r in args.serve_rates.split(",") if r]
            line["served"] = served_mode(torch, vnp, vnp_gen, rates, args.serve_seconds, args.compare_seconds)
        except Exception as e:  # noqa: BLE001
            line["served"] = {"error": repr(e)}
    if not args.no_cpu:
        line["cpu_baseline"], xc = cpu_baseline(1 << args.cpu_sample_log2)
        line["oracle_timings"] = oracle_timings(xc)
        del xc
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
