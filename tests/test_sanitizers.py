"""Address and undefined-behaviour sanitizer build of the host code that runs
on the CPU: the oracle's C reaction sums (oracle/direct.c) and the library's
host planners (batch grouping and hexagonal tessellation, csrc/plan.hip,
which holds no device code), driven by tests/sanitize/driver.cpp.  Built with
gcc / g++ for the host only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_under_sanitizers(tmp_path):
    d = str(tmp_path)
    direct = os.path.join(d, "direct.o")
    plan = os.path.join(d, "plan.o")
    exe = os.path.join(d, "driver")
    subprocess.check_call(["gcc", *SAN, "-std=c11", "-fopenmp", "-c",
                           os.path.join(ROOT, "oracle", "direct.c"), "-o", direct])
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-c",
                           os.path.join(ROOT, "paper_1702_03781_amd", "csrc", "plan.hip"), "-o", plan])
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-fopenmp", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), plan, direct, "-o", exe,
                           "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitize ok" in r.stdout
