// FP32 product kernels: one plain (one tile per workgroup) and one grouped
// (persistent workgroups walking the tiles of many problems) kernel per tile
// configuration.
#include "kernels.hpp"
#include "tile_f32.hpp"

template <int BM, int BN, int OCC>
__global__ __launch_bounds__(GEMM_THREADS, OCC) void gemm_f32_plain_kernel(TileProblem P) {
    typedef F32Cfg<BM, BN> Cfg;
    __shared__ __attribute__((aligned(16))) float lds[Cfg::LDS_FLOATS];
    const int per_split = P.tiles_m * P.tiles_n;
    int t = xcd_remap(blockIdx.x, gridDim.x);
    const int split = t / per_split;
    t -= split * per_split;
    int tm, tn;
    tile_coords(t, P.tiles_m, P.tiles_n, 8, tm, tn);
    f32_tile<Cfg>(P, tm, tn, split, lds);
}

// Locate the problem that owns global tile t (descs sorted by tile_start).
__device__ __forceinline__ int group_find(const GroupDesc *d, int count, int t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_start <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int BM, int BN, int OCC>
__global__ __launch_bounds__(GEMM_THREADS, OCC) void gemm_f32_grouped_kernel(GroupedArgs G) {
    typedef F32Cfg<BM, BN> Cfg;
    __shared__ __attribute__((aligned(16))) float lds[Cfg::LDS_FLOATS];
    for (int t = blockIdx.x; t < G.total_tiles; t += gridDim.x) {
        const int p = group_find(G.descs, G.count, t);
        const TileProblem P = G.descs[p].P;
        int tm, tn;
        tile_coords(t - G.descs[p].tile_start, P.tiles_m, P.tiles_n, 8, tm, tn);
        f32_tile<Cfg>(P, tm, tn, 0, lds);
    }
}

template <int BM, int BN, int OCC>
static hipError_t launch_plain(const TileProblem &P, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_f32_plain_kernel<BM, BN, OCC>), dim3(nwg), dim3(GEMM_THREADS), 0, s, P);
    return hipGetLastError();
}

template <int BM, int BN, int OCC>
static hipError_t launch_grouped(const GroupedArgs &G, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_f32_grouped_kernel<BM, BN, OCC>), dim3(nwg), dim3(GEMM_THREADS), 0, s, G);
    return hipGetLastError();
}

#define F32_CFG(BM, BN, OCC)                                                                  \
    {BM, BN, F32Cfg<BM, BN>::BK, 4, F32Cfg<BM, BN>::LDS_BYTES, 2,                              \
     (160 * 1024 / F32Cfg<BM, BN>::LDS_BYTES) < OCC ? (160 * 1024 / F32Cfg<BM, BN>::LDS_BYTES) \
                                                    : OCC,                                     \
     launch_plain<BM, BN, OCC>, launch_grouped<BM, BN, OCC>}

static const KernelCfg kF32Configs[] = {
    F32_CFG(256, 256, 1),
    F32_CFG(256, 128, 1),
    F32_CFG(128, 256, 1),
    F32_CFG(128, 128, 2),
    F32_CFG(128, 64, 2),
    F32_CFG(64, 128, 2),
    F32_CFG(64, 64, 4),
};

const KernelCfg *f32_configs(int *count) {
    *count = (int)(sizeof(kF32Configs) / sizeof(kF32Configs[0]));
    return kF32Configs;
}
