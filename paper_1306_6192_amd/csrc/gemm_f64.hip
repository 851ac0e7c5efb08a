// Binary64 product kernels: the plain launch for every tile configuration
// (register-staged tiles for any shape; asynchronous-copy tiles for shapes
// whose k, n and row strides are whole 16-byte chunks).
#include "kernels_impl.hpp"
#include "tile_f64.hpp"
#include "tile_lp2.hpp"

// 128x128 runs two waves per SIMD (252 VGPRs): one wave's binary64 MFMAs
// cover the other's loads, LDS staging and barrier.  Measured at 8192^3 it
// sustains 62 TFLOP/s against 58 for a 256x128 tile at one wave per SIMD and
// 61 for a 256x128 tile of eight waves.
static const KernelCfg kF64Configs[] = {
    make_cfg<F64Cfg<128, 128>, 2>(),
    make_cfg<F64Cfg<64, 64>, 4>(),
    // asynchronous-copy tiles (four-stage LDS ring of 16-double k-tiles):
    // eight waves (64 x 32 each) and four waves (64 x 64 each) on 128x128
    make_cfg<Lp2Cfg<GEMM_MODE_F64, 128, 128, 4, 2, 4>, 2, 2>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F64, 128, 128, 4>, 1, 2>(),
};

const KernelCfg *f64_configs(int *count) {
    *count = (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0]));
    return kF64Configs;
}
