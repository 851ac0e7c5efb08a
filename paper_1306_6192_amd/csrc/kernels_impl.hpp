// Kernel templates shared by every mode: the plain launch (one output tile
// per workgroup, XCD-aware tile order) and the grouped persistent launch
// (workgroups walk the tiles of many problems, each problem with one of two
// tile configurations).
#pragma once

#include "kernels.hpp"

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

// Locate the problem that owns global tile t (descriptors sorted by
// tile_start, binary search).
__device__ __forceinline__ int group_find(const GroupDesc *d, int count, int t) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].tile_start <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int A, int B> struct cmax { static constexpr int v = A > B ? A : B; };

// Persistent workgroups take tiles from a queue (one atomic increment per
// tile) over the concatenated tile lists, which the host orders from the
// costliest tile to the cheapest, so the tiles are handed out greedily,
// longest first.  Descriptor field `cfg` selects Cfg0 or Cfg1 for a problem.
// Every workgroup leaves the loop once the queue is exhausted, so the grid
// always drains; the last one out resets the queue for the next launch.
template <class Cfg0, class Cfg1, int OCC>
__global__ __launch_bounds__(Cfg0::THREADS, OCC) void gemm_grouped_kernel(GroupedArgs G) {
    static_assert(Cfg0::THREADS == Cfg1::THREADS, "one workgroup size per grouped launch");
    __shared__ __attribute__((aligned(16))) uint8_t lds[cmax<Cfg0::LDS_BYTES, Cfg1::LDS_BYTES>::v];
    __shared__ int next_tile;
    while (true) {
        if (threadIdx.x == 0) next_tile = atomicAdd(&G.counters[0], 1);
        __syncthreads();
        const int t = next_tile;
        __syncthreads();
        if (t >= G.total_tiles) break;
        const int p = group_find(G.descs, G.count, t);
        const GroupDesc &d = G.descs[p];
        const TileProblem P = d.P;
        const int local = t - d.tile_start;
        int tm, tn;
        if (d.cfg == 0) {
            tile_coords(local, P.tiles_m, P.tiles_n, 8, tm, tn);
            Cfg0::run(P, tm, tn, 0, lds);
        } else {
            tile_coords(local, P.tiles_m, P.tiles_n, 8, tm, tn);
            Cfg1::run(P, tm, tn, 0, lds);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&G.counters[1], 1) == (int)gridDim.x - 1) {
            atomicExch(&G.counters[0], 0);
            atomicExch(&G.counters[1], 0);
        }
    }
}

template <class Cfg, int OCC>
static hipError_t launch_plain_t(const TileProblem &P, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_plain_kernel<Cfg, OCC>), dim3(nwg), dim3(Cfg::THREADS), 0, s, P);
    return hipGetLastError();
}

template <class Cfg0, class Cfg1, int OCC>
static hipError_t launch_grouped_t(const GroupedArgs &G, int nwg, hipStream_t s) {
    hipLaunchKernelGGL((gemm_grouped_kernel<Cfg0, Cfg1, OCC>), dim3(nwg), dim3(Cfg0::THREADS), 0, s, G);
    return hipGetLastError();
}

// LDS of a grouped kernel: the larger of its two tiles' rings plus the
// claimed-tile word.
template <class Cfg0, class Cfg1>
constexpr int grouped_lds_bytes() {
    return cmax<Cfg0::LDS_BYTES, Cfg1::LDS_BYTES>::v + (int)sizeof(int);
}

// A grouped kernel's table entry: its resident workgroups per CU are the
// launch bound, capped by what fits in the CU's 160 KiB of LDS.
template <class Cfg0, class Cfg1, int OCC>
constexpr GroupedKernel make_grouped(int cfg0, int cfg1) {
    return GroupedKernel{{cfg0, cfg1},
                         (160 * 1024 / grouped_lds_bytes<Cfg0, Cfg1>()) < OCC
                             ? (160 * 1024 / grouped_lds_bytes<Cfg0, Cfg1>())
                             : OCC,
                         grouped_lds_bytes<Cfg0, Cfg1>(),
                         launch_grouped_t<Cfg0, Cfg1, OCC>};
}

template <class Cfg, int OCC, int CHUNK = 0, int PRESPLIT = 0>
constexpr KernelCfg make_cfg() {
    return KernelCfg{Cfg::BM, Cfg::BN, Cfg::BK, Cfg::THREADS / 64, Cfg::LDS_BYTES, Cfg::MFMA_K,
                     (160 * 1024 / Cfg::LDS_BYTES) < OCC ? (160 * 1024 / Cfg::LDS_BYTES) : OCC,
                     launch_plain_t<Cfg, OCC>, CHUNK, PRESPLIT};
}
