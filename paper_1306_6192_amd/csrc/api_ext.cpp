// C-ABI entry points of the binary64 and complex-float products and of the
// element-wise matrix addition (plain launches, no split-K, no workspace).
#include <algorithm>
#include <cstring>

#include "host.hpp"

namespace mg {

static const int64_t kMaxDimExt = (int64_t)1 << 30;

static bool overlap(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Shape, stride, pointer and overlap checks of a product whose elements are
// `es` bytes (A, B and C alike).  No HIP call, no memory access.
static int validate_ext(int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *B, int64_t ldb,
                        const void *C, int64_t ldc, size_t es) {
    if (m < 0 || n < 0 || k < 0)
        return fail(GEMM_EINVAL, "negative dimension (m=%lld n=%lld k=%lld)", (long long)m, (long long)n,
                    (long long)k);
    if (m > kMaxDimExt || n > kMaxDimExt || k > kMaxDimExt) return fail(GEMM_EUNSUPPORTED, "dimension above 2^30");
    if (lda < std::max<int64_t>(1, k)) return fail(GEMM_EINVAL, "lda=%lld < max(1,k=%lld)", (long long)lda, (long long)k);
    if (ldb < std::max<int64_t>(1, n)) return fail(GEMM_EINVAL, "ldb=%lld < max(1,n=%lld)", (long long)ldb, (long long)n);
    if (ldc < std::max<int64_t>(1, n)) return fail(GEMM_EINVAL, "ldc=%lld < max(1,n=%lld)", (long long)ldc, (long long)n);
    const bool out_empty = m == 0 || n == 0;
    if (!out_empty && !C) return fail(GEMM_EINVAL, "C is NULL for a non-empty output");
    if (!out_empty && k > 0 && (!A || !B)) return fail(GEMM_EINVAL, "A or B is NULL for a non-empty product");
    if (!out_empty && k > 0) {
        const size_t cbytes = ((size_t)(m - 1) * ldc + n) * es;
        const size_t abytes = ((size_t)(m - 1) * lda + k) * es;
        const size_t bbytes = ((size_t)(k - 1) * ldb + n) * es;
        if (overlap(C, cbytes, A, abytes) || overlap(C, cbytes, B, bbytes))
            return fail(GEMM_EINVAL, "C overlaps A or B");
    }
    return GEMM_OK;
}

// One plain launch of configuration `cfg` of family `mode` (F64 or C32).
static int enqueue_ext(int mode, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                       int64_t ldb, void *C, int64_t ldc, int cfg, hipStream_t s) {
    const size_t es = 8;   // double, or a (re, im) float pair
    if (m == 0 || n == 0) return GEMM_OK;
    if (k == 0) {
        MG_HIP(launch_zero_rows(C, ldc * (int64_t)es, (int)m, n * (int64_t)es, s));
        return GEMM_OK;
    }
    int count = 0;
    const KernelCfg *t = configs(mode, &count);
    if (!t || count == 0) return fail(GEMM_EUNSUPPORTED, "mode %d has no kernels", mode);
    if (cfg < 0 || cfg >= count) return fail(GEMM_EINVAL, "config %d out of range [0,%d)", cfg, count);
    {
        // an asynchronous-copy configuration needs whole 16-byte chunks;
        // otherwise its register-staged counterpart of the same tile runs
        gemm_problem_t p;
        memset(&p, 0, sizeof(p));
        p.mode = mode;
        p.m = m;
        p.n = n;
        p.k = k;
        p.A = A;
        p.lda = lda;
        p.B = B;
        p.ldb = ldb;
        cfg = effective_cfg(p, cfg);
    }
    const KernelCfg &kc = t[cfg];
    TileProblem P;
    memset(&P, 0, sizeof(P));
    P.A = A;
    P.B = B;
    P.C = static_cast<float *>(C);   // element type fixed by the family's tile
    P.lda = lda;
    P.ldb = ldb;
    P.ldc = ldc;
    P.m = (int32_t)m;
    P.n = (int32_t)n;
    P.k = (int32_t)k;
    P.tiles_m = (int32_t)((m + kc.bm - 1) / kc.bm);
    P.tiles_n = (int32_t)((n + kc.bn - 1) / kc.bn);
    P.splits = 1;
    P.kt_per_split = (int32_t)((k + kc.bk - 1) / kc.bk);
    P.scale = 1.f;
    const int64_t nwg = (int64_t)P.tiles_m * P.tiles_n;
    if (nwg > INT32_MAX) return fail(GEMM_EUNSUPPORTED, "too many output tiles");
    MG_HIP(kc.plain(P, (int)nwg, s));
    return GEMM_OK;
}

static int plain_ext(int mode, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                     int64_t ldb, void *C, int64_t ldc, int cfg, void *stream) {
    int rc = validate_ext(m, n, k, A, lda, B, ldb, C, ldc, 8);
    if (rc != GEMM_OK) return rc;
    if (cfg < 0) {
        int split = 1;
        tuner_choose(mode, m, n, k, &cfg, &split);
    }
    return enqueue_ext(mode, m, n, k, A, lda, B, ldb, C, ldc, cfg, (hipStream_t)stream);
}

}  // namespace mg

using namespace mg;

extern "C" {

int gemm_plain_f64(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *C, int64_t ldc, void *stream) {
    clear_error();
    return plain_ext(GEMM_MODE_F64, m, n, k, A, lda, B, ldb, C, ldc, -1, stream);
}

int gemm_plain_f64_cfg(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, int64_t ldc, int32_t cfg, void *stream) {
    clear_error();
    if (cfg < 0) return fail(GEMM_EINVAL, "config %d out of range", cfg);
    return plain_ext(GEMM_MODE_F64, m, n, k, A, lda, B, ldb, C, ldc, cfg, stream);
}

int gemm_plain_c32(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                   float *C, int64_t ldc, void *stream) {
    clear_error();
    return plain_ext(GEMM_MODE_C32, m, n, k, A, lda, B, ldb, C, ldc, -1, stream);
}

int gemm_plain_c32_cfg(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
                       int64_t ldb, float *C, int64_t ldc, int32_t cfg, void *stream) {
    clear_error();
    if (cfg < 0) return fail(GEMM_EINVAL, "config %d out of range", cfg);
    return plain_ext(GEMM_MODE_C32, m, n, k, A, lda, B, ldb, C, ldc, cfg, stream);
}

int gemm_add(int32_t dtype, int32_t subtract, int64_t m, int64_t n, const void *A, int64_t lda, const void *B,
             int64_t ldb, void *C, int64_t ldc, void *stream) {
    clear_error();
    size_t es;
    if (dtype == GEMM_MODE_F32) es = 4;
    else if (dtype == GEMM_MODE_F64) es = 8;
    else return fail(GEMM_EUNSUPPORTED, "gemm_add takes GEMM_MODE_F32 or GEMM_MODE_F64 (got %d)", dtype);
    if (m < 0 || n < 0) return fail(GEMM_EINVAL, "negative dimension (m=%lld n=%lld)", (long long)m, (long long)n);
    if (m > kMaxDimExt || n > kMaxDimExt) return fail(GEMM_EUNSUPPORTED, "dimension above 2^30");
    const int64_t minld = std::max<int64_t>(1, n);
    if (lda < minld || ldb < minld || ldc < minld)
        return fail(GEMM_EINVAL, "strides must be >= max(1, n=%lld)", (long long)n);
    if (m == 0 || n == 0) return GEMM_OK;
    if (!A || !B || !C) return fail(GEMM_EINVAL, "NULL matrix pointer");
    const size_t abytes = ((size_t)(m - 1) * lda + n) * es;
    const size_t bbytes = ((size_t)(m - 1) * ldb + n) * es;
    const size_t cbytes = ((size_t)(m - 1) * ldc + n) * es;
    // in place (C is A or B, same stride) is fine; any other overlap is not
    const bool c_is_a = C == A && ldc == lda, c_is_b = C == B && ldc == ldb;
    if ((!c_is_a && overlap(C, cbytes, A, abytes)) || (!c_is_b && overlap(C, cbytes, B, bbytes)))
        return fail(GEMM_EINVAL, "C partially overlaps A or B");
    MG_HIP(launch_ew_add((int)es, A, lda, B, ldb, C, ldc, (int)m, (int)n, subtract ? 1 : 0, (hipStream_t)stream));
    return GEMM_OK;
}

}  // extern "C"
