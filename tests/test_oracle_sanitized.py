"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with -fsanitize=address,undefined and no recovery into
a temporary directory, and the oracle's CPU pin suite runs against that build
in a child process with the ASan runtime preloaded (SAAMG_ORACLE_LIB names the
instrumented library): an out-of-bounds access, a use after free or
undefined behaviour (signed overflow, misaligned access, bad shift) aborts
the child and fails this test.  Leak detection is off: the Python
interpreter itself keeps allocations alive at exit.
"""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "saamg_oracle.c")


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("the ASan runtime is not installed")
    so = tmp_path / "libsaamg_oracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(so), SRC, "-lm"], check=True)
    env = dict(os.environ, SAAMG_ORACLE_LIB=str(so), LD_PRELOAD=libasan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    files = [f for f in files if not f.endswith("test_oracle_sanitized.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                          "-m", "not gpu", *files], env=env, cwd=ROOT, capture_output=True, text=True, timeout=1500)
    tail = (res.stdout[-4000:] + res.stderr[-4000:])
    assert res.returncode == 0, tail
    assert "passed" in res.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
