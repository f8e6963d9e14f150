"""The oracle side of the synthetic accuracy study (the tester of Sect. 2 and Fig. 1 on
stand-in inputs; Table 4 of Sect. 5 for p != 2), against the GPU results that
`bench.py --accuracy-gpu OUT` stores (exact hex strings).  Oracle arithmetic only: runs on
any host, takes hours at the paper's sizes, and is not collected by pytest.

    python tests/accuracy_study.py GPU_JSON [--part frobenius|pnorm|all] [--pa-log2 22]
                                   [--ref-cache FILE]

Frobenius: relerr (Eq. (relerr), multiples of eps) against the exact norm, for the GPU
results and the oracle's A, H, Z and Theorem 1's single accumulator on the same inputs.
p-norms: the GPU results (at the stored n) and the oracle's A_p (on the first 2^pa_log2
elements) against the binary128 references, flat (sum |x_i|^p)^(1/p) and the recursion
with the rounded exponents RN(p/2), RN(1/p).  One JSON line on stdout, progress on stderr."""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402  (the study's input definitions, STUDY_PS, STUDY_BINS)
import oracle  # noqa: E402
import vnp_gen  # noqa: E402


def histogram(v):
    h, _ = np.histogram(np.minimum(np.asarray(v, dtype=np.float64), 1e300), bins=bench.STUDY_BINS)
    return [int(c) for c in h]


def frobenius(g):
    n, seeds = g["n"], g["seeds"]
    methods = ("gpu", "A", "H", "Z", "acc")
    out = {}
    for key, gvals in g["frobenius"].items():
        dist, fmt = key.rsplit(" ", 1)
        errs = {m: [] for m in methods}
        for sd in range(seeds):
            t0 = time.time()
            x = bench.study_input(vnp_gen, dist, fmt, sd, n)
            ex = oracle.exact_nrm2(x)
            vals = {"gpu": float.fromhex(gvals[sd]), "A": oracle.nrmf(x, "A"), "H": oracle.nrmf(x, "H"),
                    "Z": oracle.nrmf(x, "Z"), "acc": oracle.nrm_acc(x)}
            for m in methods:
                errs[m].append(oracle.relerr(vals[m], ex, fmt))
            del x
            print(f"accuracy study: {key} seed {sd} ({time.time() - t0:.1f} s) " +
                  " ".join(f"{m}={errs[m][-1]:.3f}" for m in methods), file=sys.stderr, flush=True)
        out[key] = {m: {"max": round(max(v), 4), "mean": round(sum(v) / len(v), 4), "hist": histogram(v)}
                    for m, v in errs.items()}
    return {"n": n, "seeds": seeds, "bins_eps": [b if b != math.inf else "inf" for b in bench.STUDY_BINS],
            "frobenius": out}


def pnorm(g, pa_log2, cache_path=None):
    """cache_path: a JSON file of the oracle's values per (p, seed) and sizes (the binary128
    references and A_p, as hex strings): read if present, written as they are computed, so
    that new GPU results are compared again without recomputing them."""
    pn_n, pseeds = g["pnorm_n"], g["pnorm_seeds"]
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    out = {}
    for name, p in bench.STUDY_PS.items():
        e = {"gpu_flat": [], "gpu_rec": [], "A_flat": [], "A_rec": []}
        for sd in range(pseeds):
            t0 = time.time()
            key = f"{name} seed {sd} n {pn_n} pa {1 << pa_log2}"
            if key not in cache:
                x = vnp_gen.host_fill(pn_n, kind="u01", seed=sd, stream=61)
                flat, rec = sum(oracle.ref_pnorm(x, p)), sum(oracle.ref_pnorm_R(x, p))
                xs = np.ascontiguousarray(x[:1 << pa_log2])
                del x
                vals = [flat, rec, oracle.nrmp(xs, p, "A"), sum(oracle.ref_pnorm(xs, p)), sum(oracle.ref_pnorm_R(xs, p))]
                cache[key] = [float(v).hex() for v in vals]
                if cache_path:
                    with open(cache_path + ".tmp", "w") as f:
                        json.dump(cache, f)
                    os.replace(cache_path + ".tmp", cache_path)
            flat, rec, o, aflat, arec = (float.fromhex(v) for v in cache[key])
            gv = float.fromhex(g["pnorm"][name][sd])
            e["gpu_flat"].append(oracle.relerr(gv, flat, "f64"))
            e["gpu_rec"].append(oracle.relerr(gv, rec, "f64"))
            e["A_flat"].append(oracle.relerr(o, aflat, "f64"))
            e["A_rec"].append(oracle.relerr(o, arec, "f64"))
            print(f"accuracy study: p={name} seed {sd} ({time.time() - t0:.1f} s) " +
                  " ".join(f"{k}={v[-1]:.3f}" for k, v in e.items()), file=sys.stderr, flush=True)
        out[name] = {k: {"max": round(max(v), 4), "mean": round(sum(v) / len(v), 4)} for k, v in e.items()}
    return {"gpu_n": pn_n, "oracle_n": 1 << pa_log2, "seeds": pseeds, "relerr": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("gpu_json")
    ap.add_argument("--part", choices=("frobenius", "pnorm", "all"), default="all")
    ap.add_argument("--pa-log2", type=int, default=22, help="n of the oracle's A_p")
    ap.add_argument("--ref-cache", default=None, help="JSON cache of the p-norm study's oracle values")
    args = ap.parse_args()
    with open(args.gpu_json) as f:
        g = json.load(f)
    r = {}
    if args.part in ("frobenius", "all") and g.get("seeds", 0) > 0:
        r.update(frobenius(g))
    if args.part in ("pnorm", "all") and g.get("pnorm_seeds", 0) > 0:
        r["pnorm"] = pnorm(g, args.pa_log2, args.ref_cache)
    print(json.dumps({"accuracy_study": r}), flush=True)


if __name__ == "__main__":
    main()
