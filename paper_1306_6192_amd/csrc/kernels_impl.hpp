// Kernel templates shared by every mode: the plain launch (one output tile
// per workgroup, XCD-aware tile order) and the grouped persistent launch
// (tile_gs.hpp: workgroups walk host-scheduled tile lists over many
// problems, each problem with one of two tile configurations).
#pragma once

#include "kernels.hpp"
#include "tile_gs.hpp"

template <class Cfg, int OCC>
__global__ __launch_bounds__(Cfg::THREADS, OCC) void gemm_plain_kernel(TileProblem P) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[Cfg::LDS_BYTES];
    const int per_split = P.tiles_m * P.tiles_n;
    int t = xcd_remap(blockIdx.x, gridDim.x);
    const int split = t / per_split;
    t -= split * per_split;
    int tm, tn;
    tile_coords(t, P.tiles_m, P.tiles_n, 8, tm, tn);
    Cfg::run(P, tm, tn, split, lds);
}

template <int A, int B> struct cmax { static constexpr int v = A > B ? A : B; };

// The two grouped kernels of a mode (the autotuner picks one per mode on a
// mixed batch; variant 0 unless measured otherwise): resident workgroups per
// CU and depth of the register ring (k-tiles in flight: DEPTH - 1).
//   0: one 128x128 tile, three workgroups per CU, one k-tile in flight;
//   1: two tiles (128x128 and 64x64, the cost model choosing per problem),
//      two workgroups per CU, three k-tiles in flight (FP32: one in flight).
// On the 512-problem workload variant 0 measured faster: the stream is bound
// by its per-step instructions, which more resident waves overlap, and the
// second tile's registers or a deeper ring do not fit three workgroups.
constexpr int GROUPED_ONE_OCC = 3, GROUPED_ONE_DEPTH = 2;
constexpr int GROUPED_TWO_OCC = 2, GROUPED_TWO_DEPTH = 4;

template <class Cfg, int OCC>
static hipError_t launch_plain_t(const TileProblem &P, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_plain_kernel<Cfg, OCC>), dim3(nwg), dim3(Cfg::THREADS), 0, s, P);
    return hipGetLastError();
}

template <class Cfg0, class Cfg1, int OCC, int DEPTH>
static hipError_t launch_grouped_t(const GroupedArgs &G, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_grouped_stream_kernel<Cfg0, Cfg1, OCC, DEPTH>), dim3(nwg), dim3(GEMM_THREADS), 0, s,
                       G.descs, G.tiles, G.wg_first);
    return hipGetLastError();
}

// A grouped kernel's table entry: its resident workgroups per CU are the
// launch bound, capped by what fits in the CU's 160 KiB of LDS (two stages
// of the larger tile); alone0 / alone1 are the larger and the smaller plain
// configuration a problem launched on its own may take.
template <class Cfg0, class Cfg1, int OCC, int DEPTH>
constexpr GroupedKernel make_grouped(int cfg0, int cfg1, int alone0, int alone1) {
    return GroupedKernel{{cfg0, cfg1},
                         {alone0, alone1},
                         (160 * 1024 / (2 * GsRing<Cfg0, Cfg1>::STAGE)) < OCC
                             ? (160 * 1024 / (2 * GsRing<Cfg0, Cfg1>::STAGE))
                             : OCC,
                         2 * GsRing<Cfg0, Cfg1>::STAGE,
                         launch_grouped_t<Cfg0, Cfg1, OCC, DEPTH>};
}

template <class Cfg, int OCC, int CHUNK = 0, int PRESPLIT = 0>
constexpr KernelCfg make_cfg() {
    return KernelCfg{Cfg::BM, Cfg::BN, Cfg::BK, Cfg::THREADS / 64, Cfg::LDS_BYTES, Cfg::MFMA_K,
                     (160 * 1024 / Cfg::LDS_BYTES) < OCC ? (160 * 1024 / Cfg::LDS_BYTES) : OCC,
                     launch_plain_t<Cfg, OCC>, CHUNK, PRESPLIT};
}
