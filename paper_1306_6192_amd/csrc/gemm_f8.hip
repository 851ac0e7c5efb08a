// F8E4M3 product kernels: the plain launch for every tile configuration
// (register-staged tiles for any shape; asynchronous-copy tiles for shapes
// whose k, n and row strides are whole 16-byte chunks) and the grouped
// persistent launch (128x128 tiles; 128x128 or 64x64 for a problem alone).
#include "kernels_impl.hpp"
#include "tile_lp.hpp"
#include "tile_lp2.hpp"

static const KernelCfg kTable[] = {
    make_cfg<LpCfg<GEMM_MODE_F8E4M3, 256, 256>, 1>(), make_cfg<LpCfg<GEMM_MODE_F8E4M3, 256, 128>, 1>(),
    make_cfg<LpCfg<GEMM_MODE_F8E4M3, 128, 256>, 1>(), make_cfg<LpCfg<GEMM_MODE_F8E4M3, 128, 128>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F8E4M3, 128, 64>, 2>(),  make_cfg<LpCfg<GEMM_MODE_F8E4M3, 64, 128>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F8E4M3, 64, 64>, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F8E4M3, 256, 256, 4>, 1, 16>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F8E4M3, 256, 128, 4>, 1, 16>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F8E4M3, 128, 256, 4>, 1, 16>(), make_cfg<Lp2Cfg<GEMM_MODE_F8E4M3, 128, 128, 4>, 2, 16>(),
    // register-staged 128 x 128 with k-tiles of 64 (half the LDS): the
    // grouped launch's large tile (16 KB of operands per k-tile)
    make_cfg<LpCfg<GEMM_MODE_F8E4M3, 128, 128, 64>, 3>(),
};

const KernelCfg *lp_configs_f8(int *count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

static const GroupedKernel kGrouped[2] = {
    make_grouped<LpCfg<GEMM_MODE_F8E4M3, 128, 128, 64>, LpCfg<GEMM_MODE_F8E4M3, 128, 128, 64>, GROUPED_ONE_OCC,
                 GROUPED_ONE_DEPTH>(11, 11, 11, 6),
    make_grouped<LpCfg<GEMM_MODE_F8E4M3, 128, 128, 64>, LpCfg<GEMM_MODE_F8E4M3, 64, 64>, GROUPED_TWO_OCC,
                 GROUPED_TWO_DEPTH>(11, 6, 11, 6)};

const GroupedKernel *lp_grouped_f8(int variant) { return &kGrouped[variant]; }
