// Binary64 product kernels: the plain launch for every tile configuration.
#include "kernels_impl.hpp"
#include "tile_f64.hpp"

// 128x128 runs two waves per SIMD (252 VGPRs): one wave's binary64 MFMAs
// cover the other's loads, LDS staging and barrier.  Measured at 8192^3 it
// sustains 62 TFLOP/s against 58 for a 256x128 tile at one wave per SIMD and
// 61 for a 256x128 tile of eight waves.
static const KernelCfg kF64Configs[] = {
    make_cfg<F64Cfg<128, 128>, 2>(),
    make_cfg<F64Cfg<64, 64>, 4>(),
};

const KernelCfg *f64_configs(int *count) {
    *count = (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0]));
    return kF64Configs;
}
