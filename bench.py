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
                      f"O-A (R with correctly rounded hypot), {threads} threads, {dt:.2f} s"}


def extra_modes(torch, vnp, vnp_gen):
    """Throughput of the other paths (informational; the headline is DNRMF)."""
    out = {}
    try:
        n = 1 << 30
        xs = torch.empty(n, dtype=torch.float32, device="cuda")
        vnp_gen.dev_fill(xs, kind="exp", lo=-20, hi=20, seed=0)
        res = torch.empty((), dtype=torch.float32, device="cuda")
        s = torch.cuda.current_stream()
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
        del xp
    except Exception as e:  # noqa: BLE001 -- report, do not hide the headline
        out["error"] = repr(e)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=30)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy 5 times (scale of the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the multi-GPU sharding "
              "is a design, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2509_06220_amd as vnp
    import vnp_gen

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
                     "kernel_ms_mean": round(kern_ms, 4), "kernel_ms_min": round(min(per), 4),
                     "algorithmic_bytes": nbytes, "plain_read_gbs": round(read_gbs, 1)},
        "result": res.item(),
    }
    del x
    torch.cuda.empty_cache()
    if not args.no_extra:
        line["extra"] = extra_modes(torch, vnp, vnp_gen)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(1 << args.cpu_sample_log2)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
