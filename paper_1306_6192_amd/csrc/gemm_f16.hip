// F16 product kernels: the plain launch for every tile configuration
// (register-staged tiles for any shape; asynchronous-copy tiles for shapes
// whose k, n and row strides are whole 16-byte chunks) and the grouped
// persistent launch (128x128 tiles; 128x128 or 64x64 for a problem alone).
#include "kernels_impl.hpp"
#include "tile_lp.hpp"
#include "tile_lp2.hpp"

static const KernelCfg kTable[] = {
    make_cfg<LpCfg<GEMM_MODE_F16, 256, 256>, 1>(), make_cfg<LpCfg<GEMM_MODE_F16, 256, 128>, 1>(),
    make_cfg<LpCfg<GEMM_MODE_F16, 128, 256>, 1>(), make_cfg<LpCfg<GEMM_MODE_F16, 128, 128>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F16, 128, 64>, 2>(),  make_cfg<LpCfg<GEMM_MODE_F16, 64, 128>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F16, 64, 64>, 4>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 4>, 1, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 128, 4>, 1, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 128, 256, 4>, 1, 8>(), make_cfg<Lp2Cfg<GEMM_MODE_F16, 128, 128, 4>, 2, 8>(),
    // eight waves (two per SIMD): 2 x 4 (128 x 64 each) and 4 x 2 (64 x 128 each)
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 4, 2, 4>, 2, 8>(), make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 4, 4, 2>, 2, 8>(),
    // register-staged k-tiles of 32 (half the LDS): three workgroups per CU
    make_cfg<LpCfg<GEMM_MODE_F16, 128, 128, 32>, 3>(),
    // asynchronous-copy k-tiles of 64 (128-byte A rows) in two LDS stages:
    // half the barriers of the k-tile-32 ring, eight waves (2 x 4, 4 x 2) or four
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 2, 2, 4, 128>, 2, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 2, 4, 2, 128>, 2, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 256, 2, 2, 2, 128>, 1, 8>(),
    // 16x16x32 MFMA blocks (same bits as the 32x32x16 tiles): four waves
    // on 256 x 128 and 128 x 256 (one per SIMD), and 128 x 128 with k-tiles
    // of 32 (four stages) or 64 (two)
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 256, 128, 4, 2, 2, 0, 16, 16>, 1, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 128, 256, 4, 2, 2, 0, 16, 16>, 1, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 128, 128, 4, 2, 2, 0, 16, 16>, 2, 8>(),
    make_cfg<Lp2Cfg<GEMM_MODE_F16, 128, 128, 2, 2, 2, 128, 16, 16>, 2, 8>(),
};

const KernelCfg *lp_configs_f16(int *count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

static const GroupedKernel kGrouped[2] = {
    make_grouped<LpCfg<GEMM_MODE_F16, 128, 128, 32>, LpCfg<GEMM_MODE_F16, 128, 128, 32>, GROUPED_ONE_OCC,
                 GROUPED_ONE_DEPTH>(13, 13, 13, 6),
    make_grouped<LpCfg<GEMM_MODE_F16, 128, 128, 32>, LpCfg<GEMM_MODE_F16, 64, 64>, GROUPED_TWO_OCC,
                 GROUPED_TWO_DEPTH>(13, 6, 13, 6)};

const GroupedKernel *lp_grouped_f16(int variant) { return &kGrouped[variant]; }
