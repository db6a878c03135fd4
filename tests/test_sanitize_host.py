"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): the
library's building, compression, export, serialization and key map
(tests/native/host_sanitize.cpp, compiled with g++ together with the library's host
sources), and the C oracle (tests/native/oracle_sanitize.c with oracle/oracle.c). Each
program checks its own results and must also finish with no sanitizer report."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1704_02272_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _run(cmd_build, exe):
    r = subprocess.run(cmd_build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    srcs = [os.path.join(ROOT, "tests", "native", "host_sanitize.cpp")] + [
        os.path.join(CSRC, f) for f in ("builder.cpp", "capi.cpp", "serialize.cpp", "reduce.cpp")]
    out = _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, *srcs, "-o", exe], exe)
    assert "all checks passed" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    out = _run(["gcc", "-std=c11", "-fopenmp", *SAN, os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"),
                os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe], exe)
    assert "all checks passed" in out
