/*
 * CPU oracle for y = A*x (test infrastructure only).
 *
 * This file is the plain definition of the sparse matrix-vector product that
 * the paper's method computes (Introduction: y = A x with A sparse and x, y
 * dense).  The EHYB format, its partitioning and its kernels reach exactly this
 * result up to the order of floating-point additions, so the oracle is the
 * definition written out, not the method:
 *
 *   y_i = sum over the stored entries (i, j) of row i, in ascending column order,
 *         of a_ij * x_j,
 *
 * summed left to right from +0.0 in IEEE binary64 with a separate multiply and
 * add (built with -ffp-contract=off).  Rows are independent; an OpenMP loop
 * over rows changes nothing in any row's result, so the output is
 * deterministic for any thread count.
 *
 * The second routine forms s_i = sum_j |a_ij| * |x_j|, the scale of the
 * per-row error bound |y_i - yhat_i| <= tol * s_i used by the parity tests.
 *
 * Nothing here is shared with the GPU library: no header of it is included and
 * no symbol of it is referenced.  Only tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.
 */
#include <stdint.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_spmv_csr_f64(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                        const double *val, const double *x, double *y, int n_threads)
{
    if (n_rows < 0) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double prod = val[p] * x[col[p]];
            s = s + prod;
        }
        y[i] = s;
    }
    return 0;
}

int oracle_abs_scale_f64(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                         const double *val, const double *x, double *s_out, int n_threads)
{
    if (n_rows < 0) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            s = s + fabs(val[p]) * fabs(x[col[p]]);
        s_out[i] = s;
    }
    return 0;
}

/* Multi right-hand side: Y[i][r] = sum_j a_ij X[j][r], X and Y row-major
 * [n][n_rhs].  Same per-row left-to-right order as the single-vector routine,
 * one independent sum per right-hand side. */
int oracle_spmm_csr_f64(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                        const double *val, int32_t n_rhs, const double *X, double *Y,
                        int n_threads)
{
    if (n_rows < 0 || n_rhs <= 0) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        for (int32_t r = 0; r < n_rhs; ++r) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double prod = val[p] * X[(int64_t)col[p] * n_rhs + r];
                s = s + prod;
            }
            Y[i * n_rhs + r] = s;
        }
    }
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
