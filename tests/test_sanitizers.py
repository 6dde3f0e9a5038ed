"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code:
the CPU oracle (oracle/oracle.c) and the host-side C++ of the library
(Chimera graph, coupling words, threshold tables, RAO move, planted
instances: hs_host.cpp, hs_lao.cpp), each driven through every entry point by
a small program under tests/support.  Host compilers only; no GPU code is
built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUPPORT = os.path.join(ROOT, "tests", "support")
CSRC = os.path.join(ROOT, "paper_1605_03607_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "san_oracle")
    subprocess.run(["gcc", "-std=c11", *SAN, "-o", exe, os.path.join(ROOT, "oracle", "oracle.c"),
                    os.path.join(SUPPORT, "sanitize_oracle.c"), "-lm"], check=True)
    assert "ok" in _run(exe)


def test_host_library_code_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ missing")
    exe = str(tmp_path / "san_host")
    subprocess.run(["g++", "-std=c++17", *SAN, "-o", exe, os.path.join(CSRC, "hs_host.cpp"),
                    os.path.join(CSRC, "hs_lao.cpp"), os.path.join(SUPPORT, "sanitize_host.cpp"), "-lpthread"],
                   check=True)
    assert "ok" in _run(exe)
