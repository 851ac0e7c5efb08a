// Host-side registry of the compiled kernel configurations.
#pragma once

#include "common.hpp"

// Descriptor of one problem inside a grouped (persistent) launch.
struct GroupDesc {
    TileProblem P;        // splits == 1
    int32_t tile_start;   // first global tile index of this problem
    int32_t cfg;          // 0 or 1: which of the grouped kernel's two tile configurations
    int32_t pad[2];
};

struct GroupedArgs {
    const GroupDesc *descs;
    int32_t count;
    int32_t total_tiles;
};

typedef hipError_t (*PlainLaunchFn)(const TileProblem &P, int nwg, hipStream_t s);
typedef hipError_t (*GroupedLaunchFn)(const GroupedArgs &G, int nwg, hipStream_t s);

struct KernelCfg {
    int bm, bn, bk, waves, lds_bytes, mfma_k;
    int wg_per_cu;             // resident workgroups per CU (register and LDS limits)
    PlainLaunchFn plain;
    // 0: any shape.  Otherwise the configuration moves whole 16-byte chunks
    // (`chunk` elements): k, n, lda and ldb must be multiples of it and A, B
    // 16-byte aligned.
    int chunk;
};

// The grouped kernel of a mode: two tile configurations (indices into the
// mode's plain table, so a problem gets the same tiles -- and bits -- as a
// plain launch of that configuration).
struct GroupedKernel {
    int cfg_idx[2];
    int wg_per_cu;
    GroupedLaunchFn launch;
};

// Tables of the configurations compiled for each mode (defined in the
// per-mode translation units).
const KernelCfg *f32_configs(int *count);
const KernelCfg *lp_configs(int mode, int *count);
const GroupedKernel *f32_grouped();
const GroupedKernel *lp_grouped(int mode);

// Elementwise / reduction kernels (misc.hip).
hipError_t launch_fill_zero(float *C, int64_t ldc, int m, int n, hipStream_t s);
hipError_t launch_splitk_reduce(const float *ws, int64_t split_stride, int splits, float scale,
                                float *C, int64_t ldc, int m, int n, hipStream_t s);
hipError_t launch_convert_f32(const float *x, int64_t count, int to_mode, void *out, hipStream_t s);
hipError_t launch_quantize_e4m3(const float *x, int64_t count, uint8_t *q, float *scale_out,
                                uint32_t *amax_scratch, hipStream_t s);
hipError_t launch_errnorm(const float *C, int64_t ldc, const double *R, int64_t ldr, int64_t m,
                          int64_t n, double *out3, double *partials, int nparts, hipStream_t s);
