/*
 * The CPU baseline's all-core form of the oracle's product -- TEST INFRASTRUCTURE ONLY.
 *
 * y = A x exactly as oracle_csr_spmv computes it (each row summed serially in stored order,
 * one rounding per product and per sum, no floating-point contraction), with the rows shared
 * among OpenMP threads in contiguous chunks.  Each row's arithmetic is unchanged, so the
 * result equals the serial oracle's bit for bit; only the time differs.  It exists to time
 * the plain definition on every host core beside the single-core figure, and is never used
 * as a parity reference.
 */
#include <omp.h>
#include <stdint.h>

int oracle_threads_available(void) { return omp_get_max_threads(); }

/* Returns the number of threads that ran the loop. */
int oracle_csr_spmv_threads(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const double *x, double *y)
{
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(static, 4096)
        for (int64_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                double p = val[k] * x[col[k]];
                s = s + p;
            }
            y[i] = s;
        }
    }
    return used;
}

/* Same for single-precision matrix values, widened exactly as oracle_csr_spmv_f32val does. */
int oracle_csr_spmv_f32val_threads(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                                   const float *val, const double *x, double *y)
{
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(static, 4096)
        for (int64_t i = 0; i < n_rows; ++i) {
            double s = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                double p = (double)val[k] * x[col[k]];
                s = s + p;
            }
            y[i] = s;
        }
    }
    return used;
}
