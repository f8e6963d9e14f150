"""Build the gfx950 library (libvnp.so) in-tree with hipcc.

Flags: -O3, no fast-math, no implicit contraction (every fma is written explicitly),
binary32 denormals kept (the compiler default), packed-FP32 instruction selection off.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvnp.so")
SOURCES = ["vnp_nrm.hip", "vnp_batched.hip", "vnp_server.cpp", "vnp_schatten.hip"]
ARCH = os.environ.get("VNP_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
             "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs, procs = [], []
    for s in srcs:  # the translation units compile in parallel
        o = os.path.join(CSRC, os.path.basename(s) + ".o")
        lang = [] if s.endswith(".hip") else ["-x", "hip"]
        cmd = [hipcc(), *HIP_FLAGS, *lang, "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(o)
    failed = [cmd for cmd, pr in procs if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-L/opt/rocm/lib", "-lrocsolver",
           "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def build_gen(verbose: bool = False):
    gen = os.path.join(ROOT, "vnp_gen")
    dev_src, dev_lib = os.path.join(gen, "gen_dev.hip"), os.path.join(gen, "libvnp_gen_dev.so")
    cmd = [hipcc(), *HIP_FLAGS, "-shared", dev_src, "-o", dev_lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(dev_lib + ".tmp", dev_lib)
    host_src, host_lib = os.path.join(gen, "gen_host.c"), os.path.join(gen, "libvnp_gen_host.so")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", host_src, "-o",
                           host_lib + ".tmp", "-lm"])
    os.replace(host_lib + ".tmp", host_lib)
    lg_src, lg_lib = os.path.join(gen, "loadgen.cpp"), os.path.join(gen, "libvnp_loadgen.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", lg_src, "-o", lg_lib + ".tmp"])
    os.replace(lg_lib + ".tmp", lg_lib)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_gen(verbose="-v" in sys.argv)
    print(LIB)
