// FP32 product kernels: the plain launch for every tile configuration
// (register-staged tiles and asynchronous-copy tiles with 4-byte loads for
// any shape; asynchronous-copy tiles with 16-byte loads for shapes whose k, n
// and row strides are whole 16-byte chunks) and the grouped persistent launch
// (register-staged 128x128 tiles; 128x128 or 64x64 for a problem alone).
#include "kernels_impl.hpp"
#include "tile_f32.hpp"
#include "tile_lp2.hpp"

static const KernelCfg kF32Configs[] = {
    make_cfg<F32Cfg<256, 256>, 1>(),
    make_cfg<F32Cfg<256, 128>, 1>(),
    make_cfg<F32Cfg<128, 256>, 1>(),
    make_cfg<F32Cfg<128, 128>, 2>(),
    make_cfg<F32Cfg<128, 64>, 2>(),
    make_cfg<F32Cfg<64, 128>, 2>(),
    make_cfg<F32Cfg<64, 64>, 4>(),
    // eight waves (two per SIMD), 256x256 tile: waves 2 x 4 (128 x 64 each)
    // and 4 x 2 (64 x 128 each)
    make_cfg<F32Cfg<256, 256, 2, 4>, 2>(),
    make_cfg<F32Cfg<256, 256, 4, 2>, 2>(),
    make_cfg<F32Cfg<256, 128, 4, 2>, 2>(),   // eight waves, 64 x 64 each
    make_cfg<F32Cfg<128, 256, 2, 4>, 2>(),
    // asynchronous-copy tiles (four-stage LDS ring, k-tiles of 16): eight
    // waves (two per SIMD) at 2 x 4 and 4 x 2, four waves with 128 x 128
    // per wave (one per SIMD, accumulators in AGPRs), eight waves on
    // 128 x 256, four waves on 128 x 128, four waves on 256 x 128 and
    // 128 x 256
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 256, 4, 2, 4>, 2, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 256, 4, 4, 2>, 2, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 256, 4>, 1, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 256, 4, 2, 4>, 2, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 128, 4>, 2, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 128, 4>, 1, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 256, 4>, 1, 4>(),
    // register-staged k-tiles of 16 (half the LDS): three workgroups per CU
    make_cfg<F32Cfg<128, 128, 2, 2, 16>, 3>(),
    make_cfg<F32Cfg<64, 64, 2, 2, 16>, 3>(),
    // asynchronous-copy tiles with k-tiles of 32 (128-byte A rows) in two
    // LDS stages: half the barriers of the k-tile-16 ring, and the loads of
    // the next k-tile still have a whole k-tile of MFMAs to land
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 256, 2, 2, 2, 128>, 1, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 256, 128, 2, 2, 2, 128>, 1, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 256, 2, 2, 2, 128>, 1, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 128, 2, 2, 2, 128>, 2, 4>(),
    // register-staged 64 x 64 with k-tiles of 32: the smaller tile of a
    // grouped problem launched on its own
    make_cfg<F32Cfg<64, 64, 2, 2, 32>, 3>(),
    // asynchronous-copy tiles with 4-byte direct loads (one element per
    // lane): any shape, stride and alignment; four-stage LDS rings of k-tiles
    // of 16, four waves: 128 x 128 and 64 x 64
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 128, 128, 4, 2, 2, 64, 4>, 2>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F32, 64, 64, 4, 2, 2, 64, 4>, 4>(),
};

const KernelCfg *f32_configs(int *count) {
    *count = (int)(sizeof(kF32Configs) / sizeof(kF32Configs[0]));
    return kF32Configs;
}

static const GroupedKernel kF32Grouped[2] = {
    make_grouped<F32Cfg<128, 128, 2, 2, 16>, F32Cfg<128, 128, 2, 2, 16>, GROUPED_ONE_OCC, GROUPED_ONE_DEPTH>(18, 18, 18,
                                                                                                         24),
    // (the 64 x 64 tile's accumulators share the 128 x 128 tile's first
    // block; the pair runs two workgroups per CU)
    make_grouped<F32Cfg<128, 128, 2, 2, 16>, F32Cfg<64, 64, 2, 2, 32>, GROUPED_TWO_OCC, GROUPED_ONE_DEPTH>(18, 24, 18,
                                                                                                        24)};

const GroupedKernel *f32_grouped(int variant) { return &kF32Grouped[variant]; }
