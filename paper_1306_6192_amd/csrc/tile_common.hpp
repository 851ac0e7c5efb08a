// Pieces shared by the FP32 and reduced-precision tile kernels: unaligned
// 16-byte global accesses and the accumulator epilogue.
#pragma once

#include "common.hpp"

// 16 bytes from any byte address.  gfx950 runs with unaligned global access
// enabled, so this is one dwordx4 load whatever the alignment.
__device__ __forceinline__ u32x4 ld16(const void *p) {
    u32x4 v;
    __builtin_memcpy(&v, p, 16);
    return v;
}

// Store the accumulators of one wave tile to C (row stride ldc) or to a
// split-K partial slab.  MFMA 32x32 result layout: lane l, register r holds
// row 8*(r/4) + 4*(l/32) + r%4 of the block; the kernels feed lane l%32 = jj
// of accumulator block cb with output column CB*jj + cb of the wave's
// columns, so each lane stores CB consecutive floats per row.
template <class Cfg>
__device__ __forceinline__ void tile_epilogue(float *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0,
                                              float scale, const f32x16 (&acc)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const int col = n0 + wn * Cfg::TN + Cfg::CB * l32;
    const bool full_cols = col + Cfg::CB <= N;
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = m0 + wm * Cfg::TM + rb * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
            if (row >= M) continue;
            float v[Cfg::CB];
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb) v[cb] = acc[rb][cb][r] * scale;
            float *p = C + (int64_t)row * ldc + col;
            if (full_cols) {
                __builtin_memcpy(p, v, sizeof(v));
            } else {
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb)
                    if (col + cb < N) p[cb] = v[cb];
            }
        }
    }
}

// Where the epilogue of split `split` writes: C itself, or the split's
// partial slab (row stride n) in the workspace.
__device__ __forceinline__ void epilogue_target(const TileProblem &P, int split, float *&C, int64_t &ldc,
                                                float &scale) {
    if (P.splits > 1) {
        C = P.C + (int64_t)split * P.split_stride;
        ldc = P.n;
        scale = 1.f;  // the split-K reduction applies the scale once
    } else {
        C = P.C;
        ldc = P.ldc;
        scale = P.scale;
    }
}
