/* y = A x for a matrix in compressed sparse row form: the assembled-matrix
 * ("classical") baseline the paper sets matrix-free operators against
 * (Sec. 3.2.2), run on all host cores with OpenMP (static row blocks).
 *
 * TEST AND BASELINE INFRASTRUCTURE ONLY (see the oracle package docstring):
 * the benchmark times it on the oracle's own assembled tangent; nothing in the
 * library calls it.
 *
 *   n        rows
 *   indptr   n+1 row starts (int64)
 *   indices  column of every stored entry (int32)
 *   data     value of every stored entry
 *   x, y     input and output vectors (y is overwritten)
 * Returns the number of threads used. */
#include <stdint.h>
#include <omp.h>

int csr_spmv(int64_t n, const int64_t* indptr, const int32_t* indices, const double* data, const double* x,
             double* y) {
    int threads = 1;
#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t k = indptr[i]; k < indptr[i + 1]; ++k) s += data[k] * x[indices[k]];
            y[i] = s;
        }
    }
    return threads;
}
