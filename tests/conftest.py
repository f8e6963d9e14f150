import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_host_parts():
    """The oracle and the host generator are plain C: build them if missing."""
    import subprocess

    import oracle

    oracle.build()
    gen = os.path.join(ROOT, "vnp_gen", "libvnp_gen_host.so")
    src = os.path.join(ROOT, "vnp_gen", "gen_host.c")
    if not os.path.exists(gen) or os.path.getmtime(gen) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", src, "-o", gen,
                               "-lm"])
    yield
