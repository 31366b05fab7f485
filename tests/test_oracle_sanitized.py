"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every parity claim rests on the oracle, so its tests also run against a copy
built with -fsanitize=address,undefined and -fno-sanitize-recover=all (any
report aborts the process), in a child process with the ASan runtime
preloaded.  A second child makes a deliberately out-of-bounds call to show
the instrumentation is live."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["tests/test_oracle_cipher.py", "tests/test_oracle_shuffle.py", "tests/test_oracle_lcg.py",
                "tests/test_oracle_properties.py", "tests/test_oracle_stats.py"]


def _asan_env():
    lib = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not lib or not os.path.isabs(lib) or not os.path.exists(lib):
        pytest.skip("gcc's ASan runtime is not installed")
    env = dict(os.environ)
    env.update(ORACLE_SANITIZE="1", LD_PRELOAD=lib, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return env


@pytest.mark.slow
def test_oracle_tests_pass_under_asan_and_ubsan():
    env = _asan_env()
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *ORACLE_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def test_sanitizer_is_live():
    env = _asan_env()
    code = ("import numpy as np, oracle\n"
            "assert oracle._LIB.endswith('liboracle_san.so')\n"
            "a = np.arange(8, dtype=np.uint32); b = a.copy()\n"
            "oracle._load().orc_discordant_pairs_brute(a.ctypes.data, b.ctypes.data, 64)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr and "heap-buffer-overflow" in r.stderr
