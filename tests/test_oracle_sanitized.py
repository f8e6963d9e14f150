"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle's own
tests (nodes, trees, exact references, bounds, arrays, complex vectors, accumulators) run
in a child process against a build with -fsanitize=address,undefined and no recovery, so
an out-of-bounds access, a use after free, signed overflow, a misaligned access or an
invalid shift in oracle/vnp_oracle.c fails this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITE = ["tests/test_oracle_nodes.py", "tests/test_oracle_trees.py", "tests/test_oracle_acc.py",
         "tests/test_oracle_mat.py", "tests/test_oracle_complex.py", "tests/test_exact.py", "tests/test_bounds.py",
         "tests/test_oracle_schatten.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_suite_under_asan_and_ubsan():
    import oracle

    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    oracle.build_sanitized()
    env = dict(os.environ)
    env.update(VNP_ORACLE_SANITIZED="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    r = subprocess.run([sys.executable, "-m", "pytest", *SUITE, "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
