// Element-wise matrix addition and subtraction (the paper's Results section
// analyses it beside the product, Fig. 9): c_ij = a_ij + b_ij or
// a_ij - b_ij, one IEEE operation per element, for float and double
// matrices.  HBM-bound: three streams of 16-byte accesses.
//
// Launch shape: blockIdx.y walks rows (grid-stride), blockIdx.x covers a
// row in spans of 256 threads x 4 chunks of 16 bytes; each thread issues its
// eight loads before any arithmetic so that they are all in flight at once.
// The double form streams with non-temporal loads and stores (measured at
// 4096^2: 6.5 TB/s against 5.7 with ordinary ones; for float the ordinary
// ones are faster, 6.9 against 6.3 TB/s).
// C may be A or B itself (same stride): every element is read by the thread
// that writes it, before the write.
#include "kernels.hpp"
#include "tile_common.hpp"

#define EW_UNROLL 4

template <typename T>
__global__ __launch_bounds__(256) void ew_add_kernel(const T *A, int64_t lda, const T *B,
                                                     int64_t ldb, T *C, int64_t ldc, int m, int n, int subtract) {
    constexpr int V = 16 / sizeof(T);
    const int64_t ch0 = (int64_t)blockIdx.x * (256 * EW_UNROLL) + threadIdx.x;
    for (int64_t row = blockIdx.y; row < m; row += gridDim.y) {
        const T *a = A + row * lda;
        const T *b = B + row * ldb;
        T *c = C + row * ldc;
        T va[EW_UNROLL][V], vb[EW_UNROLL][V];
#pragma unroll
        for (int u = 0; u < EW_UNROLL; ++u) {
            const int64_t col = (ch0 + u * 256) * V;
            if (col + V <= n) {
                if constexpr (sizeof(T) == 8) {
                    const u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a + col));
                    const u32x4 y = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(b + col));
                    __builtin_memcpy(va[u], &x, 16);
                    __builtin_memcpy(vb[u], &y, 16);
                } else {
                    __builtin_memcpy(va[u], a + col, 16);
                    __builtin_memcpy(vb[u], b + col, 16);
                }
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    va[u][e] = col + e < n ? a[col + e] : T(0);
                    vb[u][e] = col + e < n ? b[col + e] : T(0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < EW_UNROLL; ++u) {
            const int64_t col = (ch0 + u * 256) * V;
            T vc[V];
#pragma unroll
            for (int e = 0; e < V; ++e) vc[e] = subtract ? va[u][e] - vb[u][e] : va[u][e] + vb[u][e];
            if (col + V <= n) {
                if constexpr (sizeof(T) == 8) {
                    u32x4 z;
                    __builtin_memcpy(&z, vc, 16);
                    __builtin_nontemporal_store(z, reinterpret_cast<u32x4 *>(c + col));
                } else {
                    __builtin_memcpy(c + col, vc, 16);
                }
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e)
                    if (col + e < n) c[col + e] = vc[e];
            }
        }
    }
}

hipError_t launch_ew_add(int elem_bytes, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                         int64_t ldc, int m, int n, int subtract, hipStream_t s) {
    const int V = 16 / elem_bytes;
    const int64_t chunks = ((int64_t)n + V - 1) / V;
    const int gx = (int)((chunks + 256 * EW_UNROLL - 1) / (256 * EW_UNROLL));
    const int gy = m < 65535 ? m : 65535;
    if (elem_bytes == 8)
        hipLaunchKernelGGL(ew_add_kernel<double>, dim3(gx, gy), dim3(256), 0, s, static_cast<const double *>(A), lda,
                           static_cast<const double *>(B), ldb, static_cast<double *>(C), ldc, m, n, subtract);
    else
        hipLaunchKernelGGL(ew_add_kernel<float>, dim3(gx, gy), dim3(256), 0, s, static_cast<const float *>(A), lda,
                           static_cast<const float *>(B), ldb, static_cast<float *>(C), ldc, m, n, subtract);
    return hipGetLastError();
}

// Zero an m x (row_bytes) region with row stride ld_bytes (4-byte multiples):
// the empty product (k = 0) of the binary64 and complex forms.
__global__ void zero_rows_kernel(uint32_t *C, int64_t ld_words, int m, int64_t row_words) {
    const int64_t total = (int64_t)m * row_words;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / row_words, c = i - r * row_words;
        C[r * ld_words + c] = 0u;
    }
}

hipError_t launch_zero_rows(void *C, int64_t ld_bytes, int m, int64_t row_bytes, hipStream_t s) {
    const int64_t total = (int64_t)m * (row_bytes / 4);
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(zero_rows_kernel, dim3((int)g), dim3(256), 0, s, static_cast<uint32_t *>(C), ld_bytes / 4, m,
                       row_bytes / 4);
    return hipGetLastError();
}
