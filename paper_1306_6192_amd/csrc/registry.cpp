// Mode -> kernel table dispatch for the reduced-precision forms.
#include "kernels.hpp"

const KernelCfg *lp_configs_bf16(int *count);
const KernelCfg *lp_configs_f16(int *count);
const KernelCfg *lp_configs_f8(int *count);
const KernelCfg *lp_configs_split(int *count);
const GroupedKernel *lp_grouped_bf16(int variant);
const GroupedKernel *lp_grouped_f16(int variant);
const GroupedKernel *lp_grouped_f8(int variant);
const GroupedKernel *lp_grouped_split(int variant);

const KernelCfg *lp_configs(int mode, int *count) {
    switch (mode) {
        case GEMM_MODE_BF16: return lp_configs_bf16(count);
        case GEMM_MODE_F16: return lp_configs_f16(count);
        case GEMM_MODE_F8E4M3: return lp_configs_f8(count);
        case GEMM_MODE_F32_SPLIT_BF16X3: return lp_configs_split(count);
        default: *count = 0; return nullptr;
    }
}

const GroupedKernel *lp_grouped(int mode, int variant) {
    switch (mode) {
        case GEMM_MODE_BF16: return lp_grouped_bf16(variant);
        case GEMM_MODE_F16: return lp_grouped_f16(variant);
        case GEMM_MODE_F8E4M3: return lp_grouped_f8(variant);
        case GEMM_MODE_F32_SPLIT_BF16X3: return lp_grouped_split(variant);
        default: return nullptr;
    }
}
