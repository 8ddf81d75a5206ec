"""The CPU tests of the C ABI under AddressSanitizer + UndefinedBehaviorSanitizer.

`python -m paper_1202_1773_amd.build --sanitize` builds libffst_asan.so from
the same sources with both sanitizers on the host code (argument checks,
plan and batch bookkeeping, error paths, the index helpers). This test runs
the ABI, index and C-header tests in a child process against that library
with the ASan runtime preloaded; any invalid access, overflow or undefined
behaviour aborts the child. Skipped when the sanitizer build is absent or
was built from other sources (it is a separate, slower build than
libffst.so, made on demand).
"""

import os
import subprocess
import sys

import pytest

from paper_1202_1773_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_under_asan_and_ubsan():
    if not os.path.exists(build.LIB_ASAN):
        pytest.skip("libffst_asan.so not built (python -m paper_1202_1773_amd.build --sanitize)")
    runtime = build.asan_runtime()
    if runtime is None:
        pytest.skip("no shared ASan runtime found")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": runtime,
        "FFST_LIBRARY": build.LIB_ASAN,
        # the interpreter itself is not instrumented and keeps memory until exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    tests = [os.path.join(ROOT, "tests", t) for t in ("test_abi_cpu.py", "test_index_cpu.py", "test_header_c.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                         env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    out = res.stdout + res.stderr
    if "built from other sources" in out:
        pytest.skip("libffst_asan.so is older than the sources: rebuild it with "
                    "python -m paper_1202_1773_amd.build --sanitize")
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in res.stdout
