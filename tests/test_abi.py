"""The C-ABI library loads on a machine without a GPU and exports every declared symbol;
the product path shares nothing with the oracle."""
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_function():
    vnp = pytest.importorskip("paper_2509_06220_amd")
    names = vnp.header_functions()
    assert len(names) >= 36
    L = vnp.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_host_only_info_calls():
    vnp = pytest.importorskip("paper_2509_06220_amd")
    assert vnp.version().startswith("vnp")
    assert vnp.tile_elems(vnp.F64) == 8192 and vnp.tile_elems(vnp.F32) == 16384
    assert vnp.tree_id(vnp.F64) != vnp.tree_id(vnp.F32)
    assert vnp.lib().vnp_set_launch_shape(3, 1) == -1  # not a power of two
    assert vnp.lib().vnp_set_launch_shape(0, 0) == 0


def test_product_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2509_06220_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b|vnpo_", txt), f
    so = os.path.join(pkg, "libvnp.so")
    if os.path.exists(so):
        syms = subprocess.run(["nm", "-D", so], capture_output=True, text=True).stdout
        assert "vnpo_" not in syms


def test_bench_refuses_several_gpus():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_p_domain_is_checked_before_any_device_work():
    """p <= 0, NaN, or so small that RN(1/p) exceeds 2^1000 (binary64) or overflows
    (binary32) is an invalid argument (the node of Sect. 4 is built from RN(1/p)); these
    calls return before touching the device, so a machine without a GPU can run them."""
    import ctypes

    vnp = pytest.importorskip("paper_2509_06220_amd")
    L = vnp.lib()
    fake = ctypes.c_void_p(256)  # never dereferenced: the argument check fails first
    for p in (0.0, -1.0, math.nan, 1e-310, 2.0 ** -1025, 2.0 ** -1001):
        assert L.vnp_dnrmp(1, fake, 1, p, fake, None) == -4, p
        assert L.vnp_dnrmp_batched(1, fake, 1, fake, p, fake, None) == -5, p
        assert L.vnp_dnrmp_mat(1, 1, fake, 1, p, fake, None) == -5, p
        assert L.vnp_dschatten(1, 1, fake, 1, p, fake, None) == -5, p
    for p in (0.0, math.nan, 1e-39, 2.0 ** -129):  # 1/p beyond the binary32 range
        assert L.vnp_snrmp(1, fake, 1, p, fake, None) == -4, p
        assert L.vnp_snrmp_batched(1, fake, 1, fake, p, fake, None) == -5, p
        assert L.vnp_snrmp_mat(1, 1, fake, 1, p, fake, None) == -5, p
        assert L.vnp_sschatten(1, 1, fake, 1, p, fake, None) == -5, p
    # plans check the descriptor's p in the plan's dtype
    h = ctypes.c_void_p()
    for dt, p in ((vnp.F64, 1e-310), (vnp.F32, 1e-39), (vnp.F64, -2.0)):
        d = vnp._PlanDesc(dt, p, 1, 256, None, 1, 256, 256, 0)
        assert L.vnp_plan_create(ctypes.byref(h), ctypes.byref(d), None) == -2, (dt, p)
