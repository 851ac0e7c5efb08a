// Split-BF16x3 product kernels (float32 operands split into bfloat16 hi/lo
// planes at staging).  Two planes per operand in LDS, so the largest tile is
// 256 x 128.
#include <iterator>
#include <vector>

#include "kernels_impl.hpp"
#include "tile_lp.hpp"

static const KernelCfg kTable[] = {
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 256, 128>, 1>(), make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 256>, 1>(),
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128>, 2>(), make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 64>, 2>(),
    make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 128>, 2>(),  make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 64>, 4>(),
};

const KernelCfg *lp_configs_bf16(int *count);

// The register-staged tiles above (any shape; the grouped launch uses two of
// them), then one pre-split entry per asynchronous-copy BF16 tile with
// k-tiles of 32: those run the split form as a BF16 product over interleaved
// operand copies and give the same bits (the BF16 kernels themselves live in
// the BF16 table).  A 32-k split-K grain of the split form is three such
// k-tiles of the interleaved product; a k-tile of 64 would straddle grains.
const KernelCfg *lp_configs_split(int *count) {
    static const std::vector<KernelCfg> table = [] {
        std::vector<KernelCfg> t(std::begin(kTable), std::end(kTable));
        int nb = 0;
        const KernelCfg *bf = lp_configs_bf16(&nb);
        for (int c = 0; c < nb; ++c)
            if (bf[c].chunk && bf[c].bk == 32) {
                KernelCfg k = bf[c];
                k.chunk = 0;
                k.presplit = 1;
                t.push_back(k);
            }
        return t;
    }();
    *count = (int)table.size();
    return table.data();
}

// two workgroups' launch bound, but the 128 x 128 tile's two-plane ring
// leaves room in LDS for one
static const GroupedKernel kGrouped =
    make_grouped<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128>, LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 64>, 2>(2, 5);

const GroupedKernel *lp_grouped_split() { return &kGrouped; }
