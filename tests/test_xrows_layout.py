"""Host check of the x-interleaved E-vector layout of the deterministic lattice
E^T (no GPU): each element node has its own word below the buffer size the
library allocates, and the per-node sum's indexing reaches exactly the words
of the element nodes that coincide with a lattice node.  Both run widths (the
natural p+1 and the sector-padded one) are checked.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2402_15940_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
@pytest.mark.parametrize("pad7", [7, 8])
def test_xrows_layout(tmp_path, pad7):
    exe = tmp_path / "xrows_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    f"-DPAFEM_XROWS_PAD7={pad7}", f"-I{CSRC}",
                    os.path.join(HERE, "native", "xrows_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad=0" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the HIP headers")
def test_fastdiv_matches_integer_division(tmp_path):
    """The launch-fixed divisions of the E^T sums (FastDiv) are exact on 31-bit numerators."""
    exe = tmp_path / "fastdiv_check"
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    f"-I{CSRC}", os.path.join(HERE, "native", "fastdiv_check.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad=0" in r.stdout
