"""The library's host-side C++ -- circuit builders, expression compiler,
the cutting of levels into launches and the server's admission/tick/retire
bookkeeping (paper_2510_15413_amd/csrc/netlist.h) -- built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run against a
plaintext model of the device (tests/host_netlist_main.cpp): exhaustive
4-bit predicates, select and SUM, radix compare/select/SUM, expression
trees, ragged launch sizes from 1 gate up, levels spanning server ticks
and the memory budget returning to its fixed part."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_netlist_main.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_netlists_under_sanitizers(tmp_path):
    exe = tmp_path / "host_netlist"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-Wall", "-Werror", "-o", str(exe), SRC])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "host netlist checks passed" in out.stdout
