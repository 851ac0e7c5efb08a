// The paper's two GPU product kernels, rebuilt for gfx950 as an ablation
// baseline for the matrix-core path (float32 only):
//   variant 0 -- one thread per output element, operands read from global
//                memory in the inner loop (Implementation section, Listing 3);
//   variant 1 -- 16x16 thread blocks that stage one 16x16 tile of A and one
//                of B in LDS per k-step, synchronise, do 16 multiply-adds
//                from LDS, synchronise (Listing 4).
// Each c_ij is accumulated in ascending r in float32 (fused multiply-add).
// Unlike the paper's listings these check bounds (any m, n, k) and use the
// row strides lda/ldb/ldc.
#include "host.hpp"

#define ABL_BS 16

__global__ __launch_bounds__(ABL_BS * ABL_BS) void ablation_global_kernel(const float *__restrict__ A, int64_t lda,
                                                                          const float *__restrict__ B, int64_t ldb,
                                                                          float *__restrict__ C, int64_t ldc, int m,
                                                                          int n, int k) {
    const int j = blockIdx.x * ABL_BS + threadIdx.x;
    const int i = blockIdx.y * ABL_BS + threadIdx.y;
    if (i >= m || j >= n) return;
    float acc = 0.f;
    for (int r = 0; r < k; ++r) acc = fmaf(A[(int64_t)i * lda + r], B[(int64_t)r * ldb + j], acc);
    C[(int64_t)i * ldc + j] = acc;
}

__global__ __launch_bounds__(ABL_BS * ABL_BS) void ablation_lds_kernel(const float *__restrict__ A, int64_t lda,
                                                                       const float *__restrict__ B, int64_t ldb,
                                                                       float *__restrict__ C, int64_t ldc, int m, int n,
                                                                       int k) {
    __shared__ float As[ABL_BS][ABL_BS + 1];
    __shared__ float Bs[ABL_BS][ABL_BS + 1];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int j = blockIdx.x * ABL_BS + tx;
    const int i = blockIdx.y * ABL_BS + ty;
    float acc = 0.f;
    for (int r0 = 0; r0 < k; r0 += ABL_BS) {
        As[ty][tx] = (i < m && r0 + tx < k) ? A[(int64_t)i * lda + r0 + tx] : 0.f;
        Bs[ty][tx] = (r0 + ty < k && j < n) ? B[(int64_t)(r0 + ty) * ldb + j] : 0.f;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ABL_BS; ++r) acc = fmaf(As[ty][r], Bs[r][tx], acc);
        __syncthreads();
    }
    if (i < m && j < n) C[(int64_t)i * ldc + j] = acc;
}

using namespace mg;

extern "C" int gemm_ablation(const gemm_problem_t *p, int32_t variant, void *stream) {
    clear_error();
    int rc = validate(p);
    if (rc != GEMM_OK) return rc;
    if (p->mode != GEMM_MODE_F32) return fail(GEMM_EUNSUPPORTED, "the paper's kernels are float32 only");
    if (variant != 0 && variant != 1) return fail(GEMM_EINVAL, "variant must be 0 (global) or 1 (LDS 16x16)");
    if (p->m == 0 || p->n == 0) return GEMM_OK;
    hipStream_t s = (hipStream_t)stream;
    const dim3 block(ABL_BS, ABL_BS);
    const dim3 grid((unsigned)((p->n + ABL_BS - 1) / ABL_BS), (unsigned)((p->m + ABL_BS - 1) / ABL_BS));
    if (grid.y > 65535) return fail(GEMM_EUNSUPPORTED, "m too large for the 2-D grid of the paper's kernels");
    const float *A = static_cast<const float *>(p->A);
    const float *B = static_cast<const float *>(p->B);
    if (variant == 0)
        hipLaunchKernelGGL(ablation_global_kernel, grid, block, 0, s, A, p->lda, B, p->ldb, p->C, p->ldc, (int)p->m,
                           (int)p->n, (int)p->k);
    else
        hipLaunchKernelGGL(ablation_lds_kernel, grid, block, 0, s, A, p->lda, B, p->ldb, p->C, p->ldc, (int)p->m,
                           (int)p->n, (int)p->k);
    MG_HIP(hipGetLastError());
    return GEMM_OK;
}
