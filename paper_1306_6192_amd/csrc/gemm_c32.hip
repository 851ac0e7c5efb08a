// Complex-float product kernels: the plain launch for every tile
// configuration (register-staged tiles for any shape; asynchronous-copy tiles
// for shapes whose k, n and row strides are whole 16-byte chunks).
#include "kernels_impl.hpp"
#include "tile_c32.hpp"
#include "tile_lp2.hpp"

// Two waves per SIMD, either as two 4-wave 128x128 workgroups per CU or as
// one 8-wave 256x128 workgroup: measured at 8192^3 they sustain 135 and 137
// real TFLOP/s against 131 for a 4-wave 256x128 tile (one wave per SIMD).
static const KernelCfg kC32Configs[] = {
    make_cfg<C32Cfg<128, 128>, 2>(),
    make_cfg<C32Cfg<64, 64>, 4>(),
    make_cfg<C32Cfg<256, 128, 2, 4>, 2>(),   // eight waves, 128 x 32 each
    // asynchronous-copy tiles (four-stage ring of k-tiles of 16 complex) on
    // 128x128: eight waves (64 x 32 each) and four waves (64 x 64 each)
    make_cfg<Lp2Cfg<GEMM_MODE_C32, 128, 128, 4, 2, 4>, 2, 2>(),
    make_cfg<Lp2Cfg<GEMM_MODE_C32, 128, 128, 4>, 1, 2>(),
};

const KernelCfg *c32_configs(int *count) {
    *count = (int)(sizeof(kC32Configs) / sizeof(kC32Configs[0]));
    return kC32Configs;
}
