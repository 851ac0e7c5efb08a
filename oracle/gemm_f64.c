/*
 * Reference (oracle) dense matrix product in IEEE binary64.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links this
 * file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no source with the GPU library.
 *
 * What it computes: the standard ("Cauchy") product of the paper's
 * Implementation section, equation for c_ij:
 *
 *     c_ij = sum_{r=0}^{k-1} a_ir * b_rj        0 <= i < m, 0 <= j < n
 *
 * for a row-major m x k matrix A (row stride lda) and a row-major k x n
 * matrix B (row stride ldb); C is m x n (row stride ldc).  The paper's own
 * index names (n x m times m x p) map onto ours as (n, m, p) -> (m, k, n).
 *
 * Each c_ij starts from 0.0 and accumulates its products in ascending r,
 * as in the paper's sequential C loop (Implementation section, Listing 1).
 * Every product and every sum is rounded to binary64: build with
 * -ffp-contract=off and without -ffast-math, so no fused multiply-add and no
 * reassociation can occur.  The loops visit (i, r, j) so that the innermost
 * loop walks rows of B and C contiguously; for a fixed (i, j) the sequence of
 * roundings is exactly the i-j-r one, so the result is bit-identical to the
 * textbook loop and to itself for any thread count (threads split rows i).
 *
 * k == 0 gives an all-zero C (the empty sum).  m == 0 or n == 0 touches
 * nothing.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void oracle_gemm_f64(int64_t m, int64_t n, int64_t k,
                     const double *A, int64_t lda,
                     const double *B, int64_t ldb,
                     double *C, int64_t ldc, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i) {
        double *c = C + i * ldc;
        for (int64_t j = 0; j < n; ++j) c[j] = 0.0;
        for (int64_t r = 0; r < k; ++r) {
            const double a = A[i * lda + r];
            const double *b = B + r * ldb;
            for (int64_t j = 0; j < n; ++j) c[j] = c[j] + a * b[j];
        }
    }
}

/*
 * One output element, c_ij, by the same definition and in the same order
 * (ascending r from 0.0).  Used to check sampled outputs of products too large
 * for the full oracle.  rows[t], cols[t] name the t-th requested element.
 */
void oracle_gemm_f64_sampled(int64_t count, const int64_t *rows,
                             const int64_t *cols, int64_t k,
                             const double *A, int64_t lda,
                             const double *B, int64_t ldb,
                             double *out, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t t = 0; t < count; ++t) {
        const double *a = A + rows[t] * lda;
        const double *b = B + cols[t];
        double s = 0.0;
        for (int64_t r = 0; r < k; ++r) s = s + a[r] * b[r * ldb];
        out[t] = s;
    }
}
