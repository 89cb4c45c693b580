"""CPU oracle (test infrastructure only).

Plain FP64 full-assembly reference for the partial-assembly H1 mass and
diffusion operators and their Jacobi-PCG solve.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import anything here; the GPU
library never does, and the two share no code.
"""
