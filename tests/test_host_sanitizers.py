"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The library's host side (argument checks, layout and size arithmetic, error
reporting, handle life cycle) is rebuilt with both sanitizers, GPU code taken
from the normal build, and the C-ABI tests that run without a GPU
(tests/test_abi.py) run again against it in a child process with the sanitizer
runtime preloaded.  Any report (heap or stack overflow, use after free,
undefined behaviour such as signed overflow or a misaligned access) fails the
test; the sanitizers abort at the first one.  Leak detection is off: the Python
interpreter itself keeps allocations until exit.
"""
import os
import subprocess
import sys

import pytest

from paper_1505_06900_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

DRIVER = """
import ctypes, sys
sys.path.insert(0, {root!r})
assert hasattr(ctypes.CDLL(None), "__asan_report_load8"), "sanitizer runtime not loaded"
import paper_1505_06900_amd._lib as L
L.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main([{tests!r}, "-q", "-s", "-m", "not gpu", "-p", "no:cacheprovider"]))
"""


def test_abi_host_paths_run_clean_under_asan_and_ubsan(tmp_path):
    runtime = B.sanitizer_runtime()
    if runtime is None:
        pytest.skip("no AddressSanitizer runtime in the ROCm compiler")
    if not all(os.path.exists(os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o")) for s in B.SOURCES):
        pytest.skip("the normal build's objects are missing (python -m paper_1505_06900_amd.build)")
    lib = B.build_sanitized(str(tmp_path))
    env = dict(os.environ)
    env.update(LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = DRIVER.format(root=ROOT, lib=lib, tests=os.path.join(HERE, "test_abi.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out and "failed" not in out, out[-2000:]
