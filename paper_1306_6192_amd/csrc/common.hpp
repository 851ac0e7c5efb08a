// Shared definitions of the gfx950 kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mi355gemm.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));

#define GEMM_THREADS 256
#define GEMM_WAVE 64

// Number of XCDs the hardware dispatcher deals workgroups over, round-robin.
#define GEMM_NUM_XCD 8

// Arguments of one tile walk over a single problem (plain launch) or of one
// problem inside a grouped launch.  Pointers are device pointers; strides are
// in elements.
struct TileProblem {
    const void *A;
    const void *B;
    float *C;            // output (or split-K partial slab base)
    int64_t lda, ldb, ldc;
    int32_t m, n, k;
    int32_t tiles_m, tiles_n;
    int32_t splits;          // split-K factor (1 = write C directly)
    int32_t kt_per_split;    // k tiles per split (last split may have fewer)
    int32_t vec;             // bit0: A rows 16-B loadable, bit1: B rows, bit2: C rows
    float scale;             // epilogue multiplier (FP8: scale_a*scale_b; else 1)
    int64_t split_stride;    // elements between split-K partial slabs
};

// Map a hardware workgroup id onto a logical tile id so that consecutive
// logical tiles land on the same XCD (which owns one L2), then walk tiles in
// groups of `group_m` tile rows so that the tiles co-resident on an XCD share
// A row panels and B column panels.
__device__ __forceinline__ int xcd_remap(int wg, int nwg) {
    const int q = nwg / GEMM_NUM_XCD;
    const int r = nwg % GEMM_NUM_XCD;
    const int xcd = wg % GEMM_NUM_XCD;
    const int idx = wg / GEMM_NUM_XCD;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

__device__ __forceinline__ void tile_coords(int t, int tiles_m, int tiles_n, int group_m,
                                            int &tm, int &tn) {
    const int per_group = group_m * tiles_n;
    const int g = t / per_group;
    const int first_m = g * group_m;
    const int gsz = min(tiles_m - first_m, group_m);
    const int in = t - g * per_group;
    tm = first_m + in % gsz;
    tn = in / gsz;
}
