// Operand preparation of the pre-split split-BF16x3 path: each float32
// operand becomes an interleaved bfloat16 copy in which every block of 16
// consecutive k holds the lo, hi and hi parts (A) or the hi, lo and hi parts
// (B) of those 16 k, so that one BF16 product over the 3 x k16 inner
// dimension computes, per 16-k step, lo_A hi_B, then hi_A lo_B, then
// hi_A hi_B: the three products of the compensated form in the order the
// register-staged split tile issues them (same bits).  hi = RNE_bf16(x),
// lo = RNE_bf16(x - hi), as at that tile's staging.
#include "kernels.hpp"
#include "tile_lp.hpp"

// Eight consecutive floats of row r from column c, zero at and beyond `cols`.
__device__ __forceinline__ void load8(const float *__restrict__ P, int64_t ld, int r, int c, int cols, float (&v)[8]) {
    const float *p = P + (int64_t)r * ld + c;
    if (c + 8 <= cols) {
        const u32x4 x = ld16(p), y = ld16(p + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            v[e] = __uint_as_float(x[e]);
            v[4 + e] = __uint_as_float(y[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = c + e < cols ? p[e] : 0.f;
    }
}

__device__ __forceinline__ void split8(const float (&v)[8], u32x4 &hi, u32x4 &lo) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t h0, l0, h1, l1;
        split_bf16(v[2 * e], h0, l0);
        split_bf16(v[2 * e + 1], h1, l1);
        hi[e] = h0 | (h1 << 16);
        lo[e] = l0 | (l1 << 16);
    }
}

// One thread per (row i, 8-wide k group j): A[i][8j..8j+7] -> the lo, hi, hi
// slots of its 16-k block b = j/2, half h = j%2.
__global__ void presplit_a_kernel(const float *__restrict__ A, int64_t lda, int m, int k, int k16,
                                  uint16_t *__restrict__ Ap) {
    const int groups = k16 / 8;
    const int64_t total = (int64_t)m * groups;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / groups), j = (int)(t % groups);
        float v[8];
        load8(A, lda, i, 8 * j, k, v);
        u32x4 hi, lo;
        split8(v, hi, lo);
        uint16_t *row = Ap + (int64_t)i * 3 * k16 + (int64_t)48 * (j / 2) + 8 * (j % 2);
        *reinterpret_cast<u32x4 *>(row) = lo;
        *reinterpret_cast<u32x4 *>(row + 16) = hi;
        *reinterpret_cast<u32x4 *>(row + 32) = hi;
    }
}

// One thread per (k row r, 8-wide column group c): B[r][8c..8c+7] -> rows
// 48 (r/16) + r%16 (hi), +16 (lo) and +32 (hi) of Bp.  Rows r >= k are zero.
__global__ void presplit_b_kernel(const float *__restrict__ B, int64_t ldb, int n, int k, int k16,
                                  uint16_t *__restrict__ Bp) {
    const int groups = n / 8;
    const int64_t total = (int64_t)k16 * groups;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(t / groups), c = (int)(t % groups);
        float v[8];
        if (r < k) {
            load8(B, ldb, r, 8 * c, n, v);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = 0.f;
        }
        u32x4 hi, lo;
        split8(v, hi, lo);
        uint16_t *base = Bp + ((int64_t)48 * (r / 16) + r % 16) * n + 8 * c;
        *reinterpret_cast<u32x4 *>(base) = hi;
        *reinterpret_cast<u32x4 *>(base + (int64_t)16 * n) = lo;
        *reinterpret_cast<u32x4 *>(base + (int64_t)32 * n) = hi;
    }
}

hipError_t launch_presplit(const float *A, int64_t lda, const float *B, int64_t ldb, int m, int n, int k,
                           uint16_t *Ap, uint16_t *Bp, hipStream_t s) {
    const int k16 = (k + 15) / 16 * 16;
    auto grid = [](int64_t work) {
        int64_t g = (work + 255) / 256;
        return (int)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
    };
    hipLaunchKernelGGL(presplit_a_kernel, dim3(grid((int64_t)m * (k16 / 8))), dim3(256), 0, s, A, lda, m, k, k16, Ap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(presplit_b_kernel, dim3(grid((int64_t)k16 * (n / 8))), dim3(256), 0, s, B, ldb, n, k, k16, Bp);
    return hipGetLastError();
}
