// FP32 output tile of C = A*B on gfx950 matrix cores (v_mfma_f32_32x32x2_f32).
//
// One workgroup of WM x WN waves (default 2 x 2, 256 lanes) owns a BM x BN
// tile of C and walks
// the k dimension in k-tiles of BK = 32 (or 16, half the LDS, for more
// resident workgroups):
//   HBM/L2 -> registers (16-B loads, masked at the edges)
//          -> LDS (two stages; A chunks swizzled, B rows padded, against
//             bank conflicts)
//          -> MFMA fragments -> float32 accumulators in AGPRs/VGPRs.
// The next k-tile's global loads are issued before the current k-tile's
// MFMAs, and written to the other LDS stage after them: one barrier per
// k-tile.  This is the shared-memory tiling of the paper's Listing 4
// (Implementation section: stage A and B sub-matrices in on-chip memory,
// synchronise, multiply from on-chip memory, synchronise) re-shaped for
// 64-wide waves and matrix-core instructions.
//
// MFMA operand layout (32x32x2, f32): lane l supplies A[l%32][kslot(l/32)]
// and B[kslot(l/32)][l%32]; the 32x32 result has, in lane l and register r,
// row 8*(r/4) + 4*(l/32) + r%4 and column l%32.
//
// k order: within a chunk of 8 consecutive k, MFMA step t (0..3) consumes
// k = 8c + t in lanes 0..31 and k = 8c + 4 + t in lanes 32..63, so that each
// lane reads its four A values with one 16-B LDS read.  Every configuration
// of this file visits the chunks in the same order, so the summation order of
// an output element does not depend on BM/BN (only split-K changes it).
//
// Columns: lane l%32 = jj of a wave owning TN = 32*CB columns reads the CB
// consecutive B values at column CB*jj (one LDS read of CB floats) and feeds
// value cb to the accumulator block cb; block cb, lane column jj is therefore
// output column CB*jj + cb, and the epilogue stores CB consecutive floats.
#pragma once

#include "tile_common.hpp"

template <int BM_, int BN_, int WM_ = 2, int WN_ = 2, int BK_ = 32>
struct F32Cfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_;
    static_assert(BK == 16 || BK == 32, "k-tiles of whole 8-k chunks, at most 32");
    // The unmasked copy of the k-loop for interior tiles costs registers; the
    // k-tile-16 tiles exist for three workgroups per CU (168 VGPRs), so they
    // run the masked loop only (same arithmetic either way).
    static constexpr bool INTERIOR_LOOP = BK == 32;
    static constexpr int WM = WM_, WN = WN_;          // waves along m and n
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM, TN = BN / WN;  // wave tile
    static constexpr int RB = TM / 32, CB = TN / 32;  // 32x32 blocks per wave
    // A rows are BK floats apart in LDS, their 16-byte chunks XOR-swizzled
    // by row (a_swz): the staging writes (four or eight chunks of a row per
    // lane group) and the fragment reads (one chunk of each of 16 rows per
    // 16-lane phase) both hit 64 distinct banks
    static constexpr int SA = BK;                     // LDS row stride of A (floats)
    static constexpr int SB = BN + 4;                 // LDS row stride of B (floats)
    static constexpr int A_ELEMS = BM * SA, B_ELEMS = BK * SB;
    static constexpr int STAGE = A_ELEMS + B_ELEMS;
    static constexpr int LDS_FLOATS = 2 * STAGE;
    static constexpr int LDS_BYTES = LDS_FLOATS * 4;
    static constexpr int AV = BM * BK / 4 / THREADS;  // float4 loads per thread (A)
    static constexpr int BV = BK * BN / 4 / THREADS;  // float4 loads per thread (B)
    static_assert(RB >= 1 && (CB == 1 || CB == 2 || CB == 4), "wave tile");
    static_assert(AV >= 1 && BV >= 1 && AV * THREADS * 4 == BM * BK && BV * THREADS * 4 == BK * BN,
                  "staging must cover the k-tile exactly");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
    static constexpr int MFMA_K = 2;
    // physical chunk of logical chunk c in A row r: c ^ a_swz(r).  Four
    // chunks per row (BK 16): 16 consecutive rows hold 4 of each (r mod 4)
    // class, and bits 1-2 of r give those 4 distinct chunks (8 consecutive
    // rows too: two of each (r mod 2) class).  Eight chunks (BK 32): 16 rows
    // hold 8 of each (r mod 2) class, spread by bits 1-3.  The swizzle does
    // not depend on the row's 32-row block, so a wave's fragment reads are
    // constant offsets from one per-lane base per chunk.
    __device__ static __forceinline__ int a_swz(int r) {
        if constexpr (BK == 32) return (r >> 1) & 7;
        return ((r >> 1) ^ (r >> 2)) & 3;
    }
    __device__ static void run(const TileProblem &P, int tm, int tn, int split, uint8_t *lds);
};

template <int CB> struct FVec;
template <> struct FVec<1> { typedef float T; };
template <> struct FVec<2> { typedef f32x2 T; };
template <> struct FVec<4> { typedef f32x4 T; };

// Four consecutive floats of row r starting at column c, zero outside
// [0,R) x [0,Cn).  Rows may start at any 4-byte address.
__device__ __forceinline__ f32x4 f32_load4(const float *__restrict__ P, int64_t ld, int r, int c, int R,
                                           int Cn) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r < R) {
        const float *p = P + (int64_t)r * ld + c;
        if (c + 3 < Cn) {
            const u32x4 u = ld16(p);
            v = __builtin_bit_cast(f32x4, u);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + e < Cn) v[e] = p[e];
        }
    }
    return v;
}

// CHECK = false: the caller guarantees that the whole BM x BK and BK x BN
// blocks lie inside A and B (interior tiles), so the loads need no masks.
template <class Cfg, bool CHECK = true>
__device__ __forceinline__ void f32_load_tiles(const TileProblem &P, int m0, int n0, int k0,
                                               f32x4 (&ra)[Cfg::AV], f32x4 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    const float *A = static_cast<const float *>(P.A);
    const float *B = static_cast<const float *>(P.B);
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 4);
        const int kv = (idx % (Cfg::BK / 4)) * 4;
        if constexpr (CHECK)
            ra[q] = f32_load4(A, P.lda, m0 + r, k0 + kv, P.m, P.k);
        else
            ra[q] = __builtin_bit_cast(f32x4, ld16(A + (int64_t)(m0 + r) * P.lda + k0 + kv));
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 4);
        const int cv = (idx % (Cfg::BN / 4)) * 4;
        if constexpr (CHECK)
            rb[q] = f32_load4(B, P.ldb, k0 + kr, n0 + cv, P.k, P.n);
        else
            rb[q] = __builtin_bit_cast(f32x4, ld16(B + (int64_t)(k0 + kr) * P.ldb + n0 + cv));
    }
}

template <class Cfg>
__device__ __forceinline__ void f32_store_tiles(float *stage, const f32x4 (&ra)[Cfg::AV],
                                                const f32x4 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    float *As = stage;
    float *Bs = stage + Cfg::A_ELEMS;
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 4);
        const int kv = (idx % (Cfg::BK / 4)) * 4;
        *reinterpret_cast<f32x4 *>(&As[r * Cfg::SA + 4 * ((kv / 4) ^ Cfg::a_swz(r))]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 4);
        const int cv = (idx % (Cfg::BN / 4)) * 4;
        *reinterpret_cast<f32x4 *>(&Bs[kr * Cfg::SB + cv]) = rb[q];
    }
}

template <class Cfg>
__device__ __forceinline__ void f32_compute_stage(const float *stage, f32x16 (&acc)[Cfg::RB][Cfg::CB]) {
    typedef typename FVec<Cfg::CB>::T BVec;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const int ar = wm * Cfg::TM + l32;                // row of row block 0
    const float *As = stage + ar * Cfg::SA;
    const float *Bs = stage + Cfg::A_ELEMS + (4 * g) * Cfg::SB + wn * Cfg::TN + Cfg::CB * l32;
#pragma unroll
    for (int kc = 0; kc < Cfg::BK / 8; ++kc) {
        f32x4 af[Cfg::RB];
        BVec bf[4];
#pragma unroll
        for (int rb = 0; rb < Cfg::RB; ++rb)
            af[rb] = *reinterpret_cast<const f32x4 *>(As + rb * 32 * Cfg::SA + 4 * ((2 * kc + g) ^ Cfg::a_swz(ar)));
#pragma unroll
        for (int t = 0; t < 4; ++t)
            bf[t] = *reinterpret_cast<const BVec *>(Bs + (kc * 8 + t) * Cfg::SB);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb) {
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb) {
                    float bv;
                    if constexpr (Cfg::CB == 1) bv = bf[t];
                    else bv = bf[t][cb];
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[rb][t], bv, acc[rb][cb], 0, 0, 0);
                }
            }
        }
    }
}

// One BM x BN output tile over the k-tiles of split `split`.
template <class Cfg>
__device__ __forceinline__ void f32_tile(const TileProblem &P, int tm, int tn, int split, float *lds) {
    const int m0 = tm * Cfg::BM, n0 = tn * Cfg::BN;
    const int nkt = (P.k + Cfg::BK - 1) / Cfg::BK;
    const int kt0 = split * P.kt_per_split;
    const int kt1 = min(kt0 + P.kt_per_split, nkt);

    f32x16 acc[Cfg::RB][Cfg::CB];
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < Cfg::CB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rb][cb][r] = 0.f;

    f32x4 ra[Cfg::AV], rbv[Cfg::BV];
    if (kt0 < kt1) {
        f32_load_tiles<Cfg>(P, m0, n0, kt0 * Cfg::BK, ra, rbv);
        f32_store_tiles<Cfg>(lds, ra, rbv);
    }
    __syncthreads();
    // Interior tiles (the whole tile and every k-tile inside the matrices)
    // run a loop whose loads carry no masks; edge tiles the masked one.  Both
    // do the same arithmetic in the same order.
    const bool interior = Cfg::INTERIOR_LOOP && m0 + Cfg::BM <= P.m && n0 + Cfg::BN <= P.n && kt1 * Cfg::BK <= P.k;
    if (interior) {
        for (int kt = kt0; kt < kt1; ++kt) {
            const int cur = (kt - kt0) & 1;
            const bool more = kt + 1 < kt1;
            if (more) f32_load_tiles<Cfg, false>(P, m0, n0, (kt + 1) * Cfg::BK, ra, rbv);
            f32_compute_stage<Cfg>(lds + cur * Cfg::STAGE, acc);
            if (more) f32_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, ra, rbv);
            __syncthreads();
        }
    } else {
        for (int kt = kt0; kt < kt1; ++kt) {
            const int cur = (kt - kt0) & 1;
            const bool more = kt + 1 < kt1;
            if (more) f32_load_tiles<Cfg>(P, m0, n0, (kt + 1) * Cfg::BK, ra, rbv);
            f32_compute_stage<Cfg>(lds + cur * Cfg::STAGE, acc);
            if (more) f32_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, ra, rbv);
            __syncthreads();
        }
    }

    float *C;
    int64_t ldc;
    float scale;
    epilogue_target(P, split, C, ldc, scale);
    tile_epilogue<Cfg>(C, ldc, P.m, P.n, m0, n0, scale, acc);
}

template <int BM, int BN, int WM, int WN, int BK>
__device__ __forceinline__ void F32Cfg<BM, BN, WM, WN, BK>::run(const TileProblem &P, int tm, int tn, int split,
                                                            uint8_t *lds) {
    f32_tile<F32Cfg<BM, BN, WM, WN, BK>>(P, tm, tn, split, reinterpret_cast<float *>(lds));
}
