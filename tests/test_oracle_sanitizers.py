"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): a driver exercises every exported function at tiny 32- and 64-bit
parameter sets and checks exact identities; any out-of-bounds access, leak or
undefined operation aborts the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_asan")
        cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               os.path.join(HERE, "oracle_asan_main.c"), os.path.join(ROOT, "oracle", "tfhe_oracle.c"),
               "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert r.stdout.strip() == "ok"
