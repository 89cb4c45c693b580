"""Build oracle/libcsr_spmv.so (the all-cores CPU SpMV baseline) with gcc -fopenmp.

Test infrastructure: only the benchmark's CPU-baseline leg loads it.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csr_spmv.c")
LIB = os.path.join(HERE, "libcsr_spmv.so")


def build() -> str:
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler for the CPU baseline")
    subprocess.run([cc, "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", SRC, "-o", LIB],
                   check=True)
    return LIB


if __name__ == "__main__":
    print(build())
