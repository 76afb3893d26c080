"""The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU needed).

The library's host code (argument validation, bin and tile tables, workspace layouts, plans,
error strings) is rebuilt with -fsanitize=address,undefined on the host side only, and the host
ABI tests (tests/test_lib_abi.py, tests/test_bin_tables.py) run against it in a child python with
the sanitizer runtime preloaded; any report aborts the child.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REGULAR = os.path.join(ROOT, "paper_2509_08675_amd", "libhufield.so")

pytestmark = pytest.mark.skipif(not os.path.exists(REGULAR) or not (shutil.which("hipcc") or
                                                                    os.path.exists("/opt/rocm/bin/hipcc")),
                                reason="needs hipcc and the regular build")


def test_host_abi_under_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2509_08675_amd import build as b
    if not all(os.path.exists(os.path.join(b.BUILD, os.path.basename(s) + ".o")) for s in b.sources()):
        pytest.skip("the regular build's objects are not present (_build/)")
    lib = b.build_host_asan()
    rt = b.asan_runtime()
    if rt is None:
        pytest.skip("AddressSanitizer runtime not found")
    env = dict(os.environ, LD_PRELOAD=rt, HUFIELD_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_lib_abi.py"), os.path.join(ROOT, "tests", "test_bin_tables.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert " passed" in r.stdout, out
