"""The library's host code (tables, lattice maps, division, E-vector layout)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on
the CPU (tests/native/host_checks.cpp); any invalid access or undefined
operation aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM_INCLUDE = "/opt/rocm/include"


def test_host_code_clean_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "host_checks")
    srcs = [os.path.join(HERE, "native", "host_checks.cpp"),
            os.path.join(ROOT, "paper_2402_15940_amd", "csrc", "host_setup.cpp")]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = [gxx, "-std=c++17", "-O1", "-g", *san, "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
           *srcs, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks passed" in r.stdout
