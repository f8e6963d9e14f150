"""The request server's host logic (pool, tickets, admission by copy, batching, completion,
destroy) under ThreadSanitizer on the CPU: tests/server_core_tsan.cpp drives the server core
of paper_2509_06220_amd/csrc/vnp_server_core.hpp with a CPU stand-in for the device from
six concurrent clients, and destroys a server with queued requests and a blocked waiter.
A data race, a lost or doubled ticket or a wrong result fails the test."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_server_core_under_sanitizer(tmp_path, sanitizer):
    exe = str(tmp_path / "server_core")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer", "-pthread",
           "-I", os.path.join(ROOT, "paper_2509_06220_amd", "csrc"), os.path.join(ROOT, "tests", "server_core_tsan.cpp"),
           "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "cannot find" in b.stderr and "san" in b.stderr:
        pytest.skip(f"gcc's {sanitizer} sanitizer runtime is not installed")
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66:second_deadlock_stack=1",
               ASAN_OPTIONS="halt_on_error=1:exitcode=67", UBSAN_OPTIONS="halt_on_error=1:exitcode=68:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "all checks passed" in r.stdout and "WARNING: ThreadSanitizer" not in out, out[-4000:]
