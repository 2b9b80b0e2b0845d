"""The library's host plan code (plan creation and queries, the data plan's
tables and density) built with AddressSanitizer and UndefinedBehaviorSanitizer
and run on the CPU, through tests/sanitize_host_driver.cpp: valid and invalid
configurations, every facet and band query, tunings, data plans with an empty
channel and rejected inputs.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2003_07358_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2003_07358_amd", "_build")
ROCM = "/opt/rocm"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the HIP headers")
def test_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(os.path.join(BUILD, "fhs_filters.h")):
        pytest.skip("build the library first (generates the filter header)")
    exe = tmp_path / "sanitize_host"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-I", BUILD, "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "sanitize_host_driver.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "hostmath.cpp"), os.path.join(CSRC, "data.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "0 failures" in r.stdout
