// Split-BF16x3 product kernels (float32 operands split into bfloat16 hi/lo
// planes at staging).  Two planes per operand in LDS, so the largest tile is
// 256 x 128.
#include "kernels_impl.hpp"
#include "tile_lp.hpp"

static const KernelCfg kTable[] = {
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 256, 128>, 1>(), make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 256>, 1>(),
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128>, 2>(), make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 64>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 128>, 2>(),  make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 64>, 4>(),
};

const KernelCfg *lp_configs_split(int *count) {
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

static const GroupedKernel kGrouped = {
    {2, 5}, 2, launch_grouped_t<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128>, LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 64>, 2>};

const GroupedKernel *lp_grouped_split() { return &kGrouped; }
