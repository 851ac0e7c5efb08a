// Binary64 product kernels: the plain launch for every tile configuration.
#include "kernels_impl.hpp"
#include "tile_f64.hpp"

static const KernelCfg kF64Configs[] = {
    make_cfg<F64Cfg<256, 128>, 1>(),
    make_cfg<F64Cfg<128, 128>, 1>(),
    make_cfg<F64Cfg<64, 64>, 4>(),
};

const KernelCfg *f64_configs(int *count) {
    *count = (int)(sizeof(kF64Configs) / sizeof(kF64Configs[0]));
    return kF64Configs;
}
