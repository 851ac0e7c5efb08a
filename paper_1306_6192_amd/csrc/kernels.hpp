// Host-side registry of the compiled kernel configurations.
#pragma once

#include "common.hpp"

// Descriptor of one problem inside a grouped (persistent) launch.
struct GroupDesc {
    TileProblem P;        // splits == 1
    int32_t cfg;          // 0 or 1: which of the grouped kernel's two tile configurations
    int32_t pad[3];
};

// One entry of a workgroup's tile list: descriptor index, the tile's first
// output row and column, and its number of k-tiles (at least 1).
struct GroupTile {
    int32_t p;
    int32_t m0, n0;
    int32_t nkt;
};

// A grouped launch: workgroup w computes tiles[wg_first[w] .. wg_first[w+1])
// in that order (the static schedule the host builds).
struct GroupedArgs {
    const GroupDesc *descs;
    const GroupTile *tiles;
    const int32_t *wg_first;
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
    // split-BF16x3 only: the float32 operands are first split into an
    // interleaved bfloat16 copy (A' = [lo hi hi], B' = [hi; lo; hi] per 16 k)
    // and the product runs as one BF16 product over 3 x k16 (`plain` is then
    // a BF16 kernel).  Needs n a multiple of 8; any k, strides, alignment.
    int presplit;
};

// The grouped kernel of a mode: the tile configurations its stream runs
// (indices into the mode's plain table, so a problem gets the same tiles --
// and bits -- as a plain launch of that configuration; the two are equal
// when the stream runs one), and the larger and the smaller configuration a
// problem launched on its own may take (a serving batch of one).
struct GroupedKernel {
    int cfg_idx[2];
    int alone_idx[2];
    int wg_per_cu;             // resident workgroups per CU (launch bound and LDS)
    int lds_bytes;             // LDS per workgroup
    GroupedLaunchFn launch;
};

// Tables of the configurations compiled for each mode (defined in the
// per-mode translation units).
const KernelCfg *f32_configs(int *count);
const KernelCfg *lp_configs(int mode, int *count);
const KernelCfg *f64_configs(int *count);   // binary64 (plain launches only)
const KernelCfg *c32_configs(int *count);   // complex float (plain launches only)
// Grouped kernel `variant` (0 or 1, see kernels_impl.hpp) of a mode.
const GroupedKernel *f32_grouped(int variant);
const GroupedKernel *lp_grouped(int mode, int variant);

// Elementwise / reduction kernels (misc.hip).
hipError_t launch_fill_zero(float *C, int64_t ldc, int m, int n, hipStream_t s);
hipError_t launch_fill_tuning(void *p, int64_t count, int elem_bytes, uint32_t seed, hipStream_t s);
hipError_t launch_splitk_reduce(const float *ws, int64_t split_stride, int splits, float scale,
                                float *C, int64_t ldc, int m, int n, hipStream_t s);
hipError_t launch_convert_f32(const float *x, int64_t count, int to_mode, void *out, hipStream_t s);
hipError_t launch_quantize_e4m3(const float *x, int64_t count, uint8_t *q, float *scale_out,
                                uint32_t *amax_scratch, hipStream_t s);
// Element-wise c = a + b or a - b (float or double, elem_bytes 4 or 8) and
// the zero fill of the binary64 / complex forms (ew.hip).
hipError_t launch_ew_add(int elem_bytes, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                         int64_t ldc, int m, int n, int subtract, hipStream_t s);
hipError_t launch_zero_rows(void *C, int64_t ld_bytes, int m, int64_t row_bytes, hipStream_t s);
// The interleaved bfloat16 operands of the pre-split split-BF16x3 path
// (presplit.hip): A (m x k float32, lda) -> Ap (m x 3 k16, row stride 3 k16);
// B (k x n float32, ldb) -> Bp (3 k16 x n, row stride n); k16 = k rounded up
// to 16, the padding zero.
hipError_t launch_presplit(const float *A, int64_t lda, const float *B, int64_t ldb, int m, int n, int k,
                           uint16_t *Ap, uint16_t *Bp, hipStream_t s);
hipError_t launch_errnorm(const float *C, int64_t ldc, const double *R, int64_t ldr, int64_t m,
                          int64_t n, double *out3, double *partials, int nparts, hipStream_t s);
