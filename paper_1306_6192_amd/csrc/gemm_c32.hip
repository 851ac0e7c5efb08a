// Complex-float product kernels: the plain launch for every tile
// configuration.
#include "kernels_impl.hpp"
#include "tile_c32.hpp"

static const KernelCfg kC32Configs[] = {
    make_cfg<C32Cfg<256, 128>, 1>(),
    make_cfg<C32Cfg<128, 128>, 2>(),
    make_cfg<C32Cfg<64, 64>, 4>(),
};

const KernelCfg *c32_configs(int *count) {
    *count = (int)(sizeof(kC32Configs) / sizeof(kC32Configs[0]));
    return kC32Configs;
}
