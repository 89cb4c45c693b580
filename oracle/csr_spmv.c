/*
 * All-cores CSR sparse matrix-vector product y = A x in FP64 (OpenMP over
 * rows), the CPU baseline of the operator apply.
 *
 * TEST INFRASTRUCTURE ONLY: used by the benchmark's CPU-baseline leg on the
 * matrix the oracle (oracle/fem.py) assembles; nothing in the GPU library
 * links it.  It is the plain definition of the product, y_i = sum_k
 * val[k] x[col[k]] over row i's entries in stored order.
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int csr_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void csr_spmv(int64_t nrows, const int64_t* rowptr, const int32_t* col, const double* val,
              const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nrows; ++i) {
    double acc = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * x[col[k]];
    y[i] = acc;
  }
}
