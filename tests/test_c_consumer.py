"""The C ABI from plain C: tests/c_consumer/c_consumer.c compiles with gcc
against include/bshuffle.h alone (CPU), and on the GPU it shuffles through
bs_shuffle / bs_shuffle_batched and matches the oracle."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_consumer"))
import make_c_consumer as c_build  # noqa: E402


def test_c_consumer_compiles(tmp_path):
    out = tmp_path / "c_consumer"
    c_build.build(str(out))
    assert out.exists()


@pytest.mark.gpu
def test_c_consumer_runs_on_the_gpu():
    if not os.path.exists(c_build.BIN):
        c_build.build()
    r = subprocess.run([c_build.BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c_consumer: OK" in r.stdout
