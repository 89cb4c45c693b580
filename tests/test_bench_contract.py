"""CPU checks of bench.py: the single-GPU contract, the algorithmic byte count
the roofline divides by, and that the committed HBM-traffic summary belongs
to the current kernel sources (the benchmark reports it only then)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("p,N", [(6, 33), (4, 50), (7, 64)])
def test_algorithmic_bytes(p, N):
    # quadrature data (6 FP64 words per point for diffusion, 1 for mass) plus
    # one read of x and one write of y, nothing for the computed restriction
    ne, n, q = N ** 3, p + 1, p + 2
    ndofs = (N * p + 1) ** 3
    assert bench.apply_bytes(ne, n, q, 6, ndofs, 8) == ne * q ** 3 * 48 + 16 * ndofs
    assert bench.apply_bytes(ne, n, q, 1, ndofs, 8) == ne * q ** 3 * 8 + 16 * ndofs
    assert bench.apply_bytes(ne, n, q, 6, ndofs, 4) == ne * q ** 3 * 24 + 8 * ndofs
    # the stored map adds 4 bytes per element node
    assert bench.apply_bytes(ne, n, q, 6, ndofs, 8, emap=True) == \
        bench.apply_bytes(ne, n, q, 6, ndofs, 8) + 4 * ne * n ** 3


def test_headline_bytes_value():
    # p = 6 on the 33^3 mesh: 35,937 elements, 7,880,599 dofs
    assert bench.apply_bytes(35937, 7, 8, 6, 7880599, 8) == 1009277296


def test_traffic_summary_matches_the_kernel_sources():
    t = bench.read_traffic("apply_diff_p6_fp64", bench.kernel_source_hash())
    assert t is not None, "profiles/apply_diff_p6_fp64_counters.txt is stale for these sources"
    algo = bench.apply_bytes(35937, 7, 8, 6, 7880599, 8)
    assert 1.0 <= t / algo <= 1.5
