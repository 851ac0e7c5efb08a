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

// The register-staged tiles above (any shape), then one pre-split entry per
// asynchronous-copy BF16 tile with
// k-tiles of 32: those run the split form as a BF16 product over interleaved
// operand copies and give the same bits (the BF16 kernels themselves live in
// the BF16 table).  A 32-k split-K grain of the split form is three such
// k-tiles of the interleaved product; a k-tile of 64 would straddle grains.
// Last, the register-staged 128 x 128 tile with k-tiles of 16 (the grouped
// launch's large tile).
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
        t.push_back(make_cfg<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128, 16>, 3>());
        return t;
    }();
    *count = (int)table.size();
    return table.data();
}

// The grouped launches' tiles: 128 x 128 with k-tiles of 16 (the last entry
// of the table above) and, in variant 1, 64 x 64; a problem launched on its
// own takes either.
const GroupedKernel *lp_grouped_split(int variant) {
    static const GroupedKernel k[2] = {
        [] {
            GroupedKernel g = make_grouped<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128, 16>,
                                           LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128, 16>, GROUPED_ONE_OCC,
                                           GROUPED_ONE_DEPTH>(0, 0, 0, 5);
            int n = 0;
            lp_configs_split(&n);
            g.cfg_idx[0] = g.cfg_idx[1] = g.alone_idx[0] = n - 1;
            return g;
        }(),
        [] {
            GroupedKernel g = make_grouped<LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 128, 128, 16>,
                                           LpCfg<GEMM_MODE_F32_SPLIT_BF16X3, 64, 64>, GROUPED_TWO_OCC,
                                           GROUPED_TWO_DEPTH>(0, 5, 0, 5);
            int n = 0;
            lp_configs_split(&n);
            g.cfg_idx[0] = g.alone_idx[0] = n - 1;
            return g;
        }()};
    return &k[variant];
}
