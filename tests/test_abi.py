"""The C-ABI library loads on a machine without a GPU and exports every declared symbol;
the product path shares nothing with the oracle."""
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
