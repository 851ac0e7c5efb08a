// FP32 product kernels: the plain launch for every tile configuration and
// the grouped persistent launch (128x128 and 64x64 tiles).
#include "kernels_impl.hpp"
#include "tile_f32.hpp"

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
};

const KernelCfg *f32_configs(int *count) {
    *count = (int)(sizeof(kF32Configs) / sizeof(kF32Configs[0]));
    return kF32Configs;
}

static const GroupedKernel kF32Grouped = {
    {3, 6}, 2, launch_grouped_t<F32Cfg<128, 128>, F32Cfg<64, 64>, 2>};

const GroupedKernel *f32_grouped() { return &kF32Grouped; }
