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

/*
 * Compensated ("double-double") product for checking a binary64 GPU product.
 *
 * A binary64 result cannot be checked against a binary64 loop whose own
 * rounding error is of the same size, so this function evaluates the same
 * definition, c_ij = sum_r a_ir b_rj in ascending r, with the compensated dot
 * product Dot2 of Ogita, Rump and Oishi ("Accurate sum and dot product",
 * SIAM J. Sci. Comput. 26(6), 2005, Algorithm 3.5): every product is split
 * exactly into a sum of two doubles (Dekker's TwoProduct, with Veltkamp's
 * splitting, so no fused multiply-add is needed), every running sum is split
 * exactly (Knuth's TwoSum), and the rounding errors are summed on the side and
 * added back at the end.  The result is as accurate as if computed in twice
 * the working precision and then rounded:
 *
 *     |res - c| <= u |c| + gamma_k^2 sum_r |a_ir b_rj|,   u = 2^-53,
 *     gamma_k = k u / (1 - k u)
 *
 * (their Proposition 3.5), valid while no product or sum under/overflows and
 * inputs stay below 2^996 in magnitude (the splitting constant must not
 * overflow).
 */
static inline void two_sum(double a, double b, double *s, double *e)
{
    const double x = a + b;
    const double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void split27(double a, double *hi, double *lo)
{
    const double c = 134217729.0 * a;   /* 2^27 + 1 */
    const double h = c - (c - a);
    *hi = h;
    *lo = a - h;
}

static inline void two_prod(double a, double b, double *p, double *e)
{
    double ah, al, bh, bl;
    const double x = a * b;
    split27(a, &ah, &al);
    split27(b, &bh, &bl);
    *e = al * bl - (((x - ah * bh) - al * bh) - ah * bl);
    *p = x;
}

static double dot2_strided(const double *a, const double *b, int64_t ldb, int64_t k)
{
    double p = 0.0, s = 0.0;
    for (int64_t r = 0; r < k; ++r) {
        double h, e, q;
        two_prod(a[r], b[r * ldb], &h, &e);
        two_sum(p, h, &p, &q);
        s = s + (q + e);
    }
    return p + s;
}

void oracle_gemm_dot2(int64_t m, int64_t n, int64_t k,
                      const double *A, int64_t lda,
                      const double *B, int64_t ldb,
                      double *C, int64_t ldc, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            C[i * ldc + j] = dot2_strided(A + i * lda, B + j, ldb, k);
}

void oracle_gemm_dot2_sampled(int64_t count, const int64_t *rows,
                              const int64_t *cols, int64_t k,
                              const double *A, int64_t lda,
                              const double *B, int64_t ldb,
                              double *out, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t t = 0; t < count; ++t)
        out[t] = dot2_strided(A + rows[t] * lda, B + cols[t], ldb, k);
}

/*
 * Complex product (the paper's Results section times float, double and
 * complex matrices; Table 2).  Operands are interleaved (re, im) pairs of
 * binary64, strides in complex elements.  Each term a_ir b_rj is the complex
 * product (ar br - ai bi) + i (ar bi + ai br), every product and sum rounded
 * to binary64, and c_ij accumulates the terms in ascending r from 0 + 0i,
 * real and imaginary parts separately.
 */
static void cdot_strided(const double *a, const double *b, int64_t ldb, int64_t k,
                         double *re, double *im)
{
    double sr = 0.0, si = 0.0;
    for (int64_t r = 0; r < k; ++r) {
        const double ar = a[2 * r], ai = a[2 * r + 1];
        const double br = b[2 * r * ldb], bi = b[2 * r * ldb + 1];
        const double tr = ar * br - ai * bi;
        const double ti = ar * bi + ai * br;
        sr = sr + tr;
        si = si + ti;
    }
    *re = sr;
    *im = si;
}

void oracle_gemm_c128(int64_t m, int64_t n, int64_t k,
                      const double *A, int64_t lda,
                      const double *B, int64_t ldb,
                      double *C, int64_t ldc, int nthreads)
{
    if (m <= 0 || n <= 0) return;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            cdot_strided(A + 2 * i * lda, B + 2 * j, ldb, k,
                         &C[2 * (i * ldc + j)], &C[2 * (i * ldc + j) + 1]);
}

void oracle_gemm_c128_sampled(int64_t count, const int64_t *rows,
                              const int64_t *cols, int64_t k,
                              const double *A, int64_t lda,
                              const double *B, int64_t ldb,
                              double *out, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t t = 0; t < count; ++t)
        cdot_strided(A + 2 * rows[t] * lda, B + 2 * cols[t], ldb, k,
                     &out[2 * t], &out[2 * t + 1]);
}
