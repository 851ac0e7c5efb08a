// Reduced-precision output tile of C = A*B on gfx950 matrix cores:
//   BF16 / F16        v_mfma_f32_32x32x16_{bf16,f16}, k-tile 64
//   FP8 E4M3          v_mfma_f32_32x32x64_f8f6f4 (no block scaling), k-tile 128
//   split-BF16x3      three v_mfma_f32_32x32x16_bf16 per step on float32
//                     inputs split at staging into hi = RNE_bf16(x) and
//                     lo = RNE_bf16(x - hi): acc += hiA hiB + hiA loB + loA hiB
// All accumulate in float32.
//
// Structure (same as the FP32 tile): 256-lane workgroup, 2 x 2 waves, two LDS
// stages, the next k-tile's global loads in flight during the current k-tile's
// MFMAs, one barrier per k-tile.
//
// Operand layout.  These MFMAs take, per lane, several consecutive-k values of
// one A row (lane l: row l%32) and of one B column (lane l: column l%32); the
// two lane halves (l/32) hold two disjoint k-groups, A and B alike.  A is
// row-major (k contiguous) in HBM, so an A row is staged as is.  B is
// row-major k x n (n contiguous), so the staging transposes it in registers:
// each thread loads TKB rows of 16 bytes (VN columns) and writes VN LDS rows
// of TKB consecutive-k elements ("B^T" rows).  Lanes of one LDS write cover
// one B^T row, so those writes are free of bank conflicts, and the global
// loads of a wave cover whole row segments of B.
//
// Column permutation: as in the FP32 tile, lane jj of accumulator block cb
// computes output column CB*jj + cb of the wave's columns, so the epilogue
// stores CB consecutive floats per lane.  The B^T row of wave-local column
// n = CB*jj + cb is stored at LDS row 32*cb + jj, which makes every fragment
// read a run of consecutive LDS rows (conflict-free with the padded stride).
#pragma once

#include "tile_common.hpp"

template <int MODE> struct LpTraits;
template <> struct LpTraits<GEMM_MODE_BF16> {
    static constexpr int IN_ESZ = 2, BK = 64, PLANES = 1, ROW = 128, KCH = 16, VB = 16;
};
template <> struct LpTraits<GEMM_MODE_F16> {
    static constexpr int IN_ESZ = 2, BK = 64, PLANES = 1, ROW = 128, KCH = 16, VB = 16;
};
template <> struct LpTraits<GEMM_MODE_F8E4M3> {
    static constexpr int IN_ESZ = 1, BK = 128, PLANES = 1, ROW = 128, KCH = 64, VB = 32;
};
template <> struct LpTraits<GEMM_MODE_F32_SPLIT_BF16X3> {
    static constexpr int IN_ESZ = 4, BK = 32, PLANES = 2, ROW = 64, KCH = 16, VB = 16;
};

// BK_ may halve the mode's k-tile (half the LDS, for more resident
// workgroups); the MFMA k-steps and their order are the same.
template <int MODE_, int BM_, int BN_, int BK_ = LpTraits<MODE_>::BK>
struct LpCfg {
    typedef LpTraits<MODE_> T;
    static constexpr int MODE = MODE_;
    static constexpr int BM = BM_, BN = BN_, BK = BK_;
    static constexpr int ROW = T::ROW / (T::BK / BK);   // bytes of a staged LDS row per plane
    static_assert(BK == T::BK || 2 * BK == T::BK, "the mode's k-tile or half of it");
    static constexpr int WM = 2, WN = 2;
    static constexpr int THREADS = GEMM_THREADS;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int RB = TM / 32, CB = TN / 32;
    static constexpr int RS = ROW + 16;          // padded LDS row stride in bytes (odd multiple of 16)
    // BF16 / F16 / FP8: A rows unpadded, their 16-byte chunks XOR-swizzled
    // by row (a_swz), so that the staging writes (several chunks of a few
    // rows per 16-lane phase) and the fragment reads (one chunk of each of
    // 16 rows per read) both hit 64 distinct banks; the padded stride puts
    // the rows of one staging phase on overlapping banks.  Split-BF16x3
    // (two planes of 8-byte pieces) keeps RS.
    static constexpr bool SWZ_A = T::PLANES == 1;
    static constexpr int RSA = SWZ_A ? ROW : RS;  // LDS row stride of A in bytes
    __device__ static __forceinline__ int a_swz(int r) {
        if constexpr (ROW / 16 == 8) return (r >> 1) & 7;
        return ((r >> 1) ^ (r >> 2)) & 3;
    }
    static constexpr int PLANE_A = BM * RSA, PLANE_B = BN * RS;
    static constexpr int A_BYTES = T::PLANES * PLANE_A, B_BYTES = T::PLANES * PLANE_B;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int LDS_BYTES = 2 * STAGE;
    static constexpr int VPR = BK * T::IN_ESZ / 16;        // 16-B global vectors per A row
    static constexpr int AV = BM * VPR / GEMM_THREADS;     // A vectors per thread
    static constexpr int VN = 16 / T::IN_ESZ;              // B columns per 16-B global vector
    static constexpr int NBLK = BN / VN;                   // column blocks of B per k-tile
    static constexpr int TKB = BK * NBLK / GEMM_THREADS;   // k rows per thread's B block
    static constexpr int KBLK = BK / TKB;                  // k blocks per k-tile
    static constexpr int MFMA_K = T::KCH;
    static_assert((RS / 16) % 2 == 1, "row stride must be an odd multiple of 16 bytes");
    static_assert(RB >= 1 && (CB == 1 || CB == 2 || CB == 4), "wave tile");
    static_assert(AV >= 1 && AV * GEMM_THREADS == BM * VPR, "A staging");
    static_assert(TKB >= 2 && TKB * KBLK == BK && KBLK * NBLK == GEMM_THREADS, "B staging");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
    __device__ static void run(const TileProblem &P, int tm, int tn, int split, uint8_t *lds);
};

// ---------------------------------------------------------------------------
// Global loads (zero outside the matrix).  Elements of ESZ bytes; a row
// segment of 16 bytes starting at element column c of row r.
template <int ESZ>
__device__ __forceinline__ u32x4 lp_load16(const uint8_t *__restrict__ base, int64_t ld, int r, int c, int R,
                                           int Cn) {
    constexpr int N = 16 / ESZ;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (r < R) {
        const uint8_t *p = base + ((int64_t)r * ld + c) * ESZ;
        if (c + N <= Cn) {
            v = ld16(p);
        } else {
            uint8_t b[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) b[i] = 0;
#pragma unroll
            for (int e = 0; e < N; ++e)
                if (c + e < Cn) {
#pragma unroll
                    for (int i = 0; i < ESZ; ++i) b[e * ESZ + i] = p[e * ESZ + i];
                }
            __builtin_memcpy(&v, b, 16);
        }
    }
    return v;
}

// float32 -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// hi = RNE_bf16(x), lo = RNE_bf16(x - hi); x - hi is exact in float32.
__device__ __forceinline__ void split_bf16(float x, uint32_t &hi, uint32_t &lo) {
    hi = bf16_rne_bits(x);
    const float r = x - __uint_as_float(hi << 16);
    lo = bf16_rne_bits(r);
}

// LDS row of the B^T row holding wave-tile-local column n (see the column
// permutation above).
template <class Cfg>
__device__ __forceinline__ int bt_row(int n) {
    const int wn = n / Cfg::TN, nn = n % Cfg::TN;
    return wn * Cfg::TN + (nn % Cfg::CB) * 32 + nn / Cfg::CB;
}

template <class Cfg>
struct LpStage {
    u32x4 a[Cfg::AV];
    u32x4 b[Cfg::TKB];
};

template <class Cfg>
__device__ __forceinline__ void lp_load_tiles(const TileProblem &P, int m0, int n0, int k0, LpStage<Cfg> &R) {
    constexpr int ESZ = Cfg::T::IN_ESZ;
    const int tid = threadIdx.x;
    const uint8_t *A = static_cast<const uint8_t *>(P.A);
    const uint8_t *B = static_cast<const uint8_t *>(P.B);
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * GEMM_THREADS;
        const int r = idx / Cfg::VPR;
        const int c = (idx % Cfg::VPR) * (16 / ESZ);
        R.a[q] = lp_load16<ESZ>(A, P.lda, m0 + r, k0 + c, P.m, P.k);
    }
    const int kb = tid % Cfg::KBLK, nb = tid / Cfg::KBLK;
#pragma unroll
    for (int e = 0; e < Cfg::TKB; ++e)
        R.b[e] = lp_load16<ESZ>(B, P.ldb, k0 + kb * Cfg::TKB + e, n0 + nb * Cfg::VN, P.k, P.n);
}

// Element c (of width W bits) of a 16-byte row vector.
template <int W>
__device__ __forceinline__ uint32_t lane_elem(const u32x4 &v, int c) {
    constexpr int PER = 32 / W;
    return (v[c / PER] >> ((c % PER) * W)) & ((1u << W) - 1u);
}

template <class Cfg>
__device__ __forceinline__ void lp_store_tiles(uint8_t *stage, const LpStage<Cfg> &R) {
    constexpr int MODE = Cfg::MODE;
    const int tid = threadIdx.x;
    uint8_t *As = stage;
    uint8_t *Bs = stage + Cfg::A_BYTES;
    // ---- A: row segments as they are (split: converted to two planes)
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * GEMM_THREADS;
        const int r = idx / Cfg::VPR;
        const int v = idx % Cfg::VPR;
        if constexpr (MODE == GEMM_MODE_F32_SPLIT_BF16X3) {
            uint32_t h[4], l[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) split_bf16(__uint_as_float(R.a[q][e]), h[e], l[e]);
            const u32x2 hv = {h[0] | (h[1] << 16), h[2] | (h[3] << 16)};
            const u32x2 lv = {l[0] | (l[1] << 16), l[2] | (l[3] << 16)};
            *reinterpret_cast<u32x2 *>(As + r * Cfg::RSA + v * 8) = hv;
            *reinterpret_cast<u32x2 *>(As + Cfg::PLANE_A + r * Cfg::RSA + v * 8) = lv;
        } else if constexpr (Cfg::SWZ_A) {
            *reinterpret_cast<u32x4 *>(As + r * Cfg::RSA + 16 * (v ^ Cfg::a_swz(r))) = R.a[q];
        } else {
            *reinterpret_cast<u32x4 *>(As + r * Cfg::RSA + v * 16) = R.a[q];
        }
    }
    // ---- B: transpose the thread's TKB x VN block into VN B^T rows
    const int kb = tid % Cfg::KBLK, nb = tid / Cfg::KBLK;
    constexpr int TKB = Cfg::TKB;
#pragma unroll
    for (int c = 0; c < Cfg::VN; ++c) {
        const int row = bt_row<Cfg>(nb * Cfg::VN + c);
        if constexpr (MODE == GEMM_MODE_F32_SPLIT_BF16X3) {
            uint32_t hw[TKB / 2], lw[TKB / 2];
#pragma unroll
            for (int p = 0; p < TKB / 2; ++p) {
                uint32_t h0, l0, h1, l1;
                split_bf16(__uint_as_float(R.b[2 * p][c]), h0, l0);
                split_bf16(__uint_as_float(R.b[2 * p + 1][c]), h1, l1);
                hw[p] = h0 | (h1 << 16);
                lw[p] = l0 | (l1 << 16);
            }
            uint8_t *dh = Bs + row * Cfg::RS + kb * TKB * 2;
            __builtin_memcpy(dh, hw, sizeof(hw));
            __builtin_memcpy(dh + Cfg::PLANE_B, lw, sizeof(lw));
        } else if constexpr (Cfg::T::IN_ESZ == 2) {
            uint32_t w[TKB / 2];
#pragma unroll
            for (int p = 0; p < TKB / 2; ++p)
                w[p] = lane_elem<16>(R.b[2 * p], c) | (lane_elem<16>(R.b[2 * p + 1], c) << 16);
            __builtin_memcpy(Bs + row * Cfg::RS + kb * TKB * 2, w, sizeof(w));
        } else {  // bytes
            uint8_t w[TKB];
#pragma unroll
            for (int e = 0; e < TKB; ++e) w[e] = (uint8_t)lane_elem<8>(R.b[e], c);
            __builtin_memcpy(Bs + row * Cfg::RS + kb * TKB, w, sizeof(w));
        }
    }
}

template <class Cfg>
__device__ __forceinline__ void lp_compute_stage(const uint8_t *stage, f32x16 (&acc)[Cfg::RB][Cfg::CB]) {
    constexpr int MODE = Cfg::MODE;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const int ar = wm * Cfg::TM + l32;             // A row of row block 0
    const uint8_t *As = stage + ar * Cfg::RSA + (Cfg::SWZ_A ? 0 : g * Cfg::T::VB);
    const uint8_t *Bs = stage + Cfg::A_BYTES + (wn * Cfg::TN + l32) * Cfg::RS + g * Cfg::T::VB;
    constexpr int CHUNK_BYTES = 2 * Cfg::T::VB;   // bytes of one MFMA k-step in a row
#pragma unroll
    for (int kc = 0; kc < Cfg::ROW / CHUNK_BYTES; ++kc) {
        if constexpr (MODE == GEMM_MODE_F8E4M3) {
            i32x8 af[Cfg::RB], bf[Cfg::CB];
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb) {
                // the lane's two chunks: 4 kc + 2 g and the next
                const uint8_t *p = As + rb * 32 * Cfg::RSA;
                const int c0 = 4 * kc + 2 * g;
                const u32x4 lo = *reinterpret_cast<const u32x4 *>(
                    p + (Cfg::SWZ_A ? 16 * (c0 ^ Cfg::a_swz(ar)) : kc * CHUNK_BYTES));
                const u32x4 hi = *reinterpret_cast<const u32x4 *>(
                    p + (Cfg::SWZ_A ? 16 * ((c0 + 1) ^ Cfg::a_swz(ar)) : kc * CHUNK_BYTES + 16));
                af[rb] = (i32x8){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                                 (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb) {
                const uint8_t *p = Bs + cb * 32 * Cfg::RS + kc * CHUNK_BYTES;
                const u32x4 lo = *reinterpret_cast<const u32x4 *>(p);
                const u32x4 hi = *reinterpret_cast<const u32x4 *>(p + 16);
                bf[cb] = (i32x8){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                                 (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[rb], bf[cb], acc[rb][cb], 0,
                                                                                 0, 0, 0, 0, 0);
        } else {
            u32x4 af[Cfg::RB], bf[Cfg::CB];
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb)
                af[rb] = *reinterpret_cast<const u32x4 *>(
                    As + rb * 32 * Cfg::RSA +
                    (Cfg::SWZ_A ? 16 * ((2 * kc + g) ^ Cfg::a_swz(ar)) : kc * CHUNK_BYTES));
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb)
                bf[cb] = *reinterpret_cast<const u32x4 *>(Bs + cb * 32 * Cfg::RS + kc * CHUNK_BYTES);
            if constexpr (MODE == GEMM_MODE_F32_SPLIT_BF16X3) {
                u32x4 al[Cfg::RB], bl[Cfg::CB];
#pragma unroll
                for (int rb = 0; rb < Cfg::RB; ++rb)
                    al[rb] = *reinterpret_cast<const u32x4 *>(As + Cfg::PLANE_A + rb * 32 * Cfg::RSA +
                                                              kc * CHUNK_BYTES);
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb)
                    bl[cb] = *reinterpret_cast<const u32x4 *>(Bs + Cfg::PLANE_B + cb * 32 * Cfg::RS +
                                                              kc * CHUNK_BYTES);
#pragma unroll
                for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < Cfg::CB; ++cb) {
                        const bf16x8 ah = __builtin_bit_cast(bf16x8, af[rb]);
                        const bf16x8 alo = __builtin_bit_cast(bf16x8, al[rb]);
                        const bf16x8 bh = __builtin_bit_cast(bf16x8, bf[cb]);
                        const bf16x8 blo = __builtin_bit_cast(bf16x8, bl[cb]);
                        f32x16 c = acc[rb][cb];
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bh, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blo, c, 0, 0, 0);
                        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
                        acc[rb][cb] = c;
                    }
            } else if constexpr (MODE == GEMM_MODE_BF16) {
#pragma unroll
                for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < Cfg::CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, af[rb]), __builtin_bit_cast(bf16x8, bf[cb]), acc[rb][cb], 0,
                            0, 0);
            } else {
#pragma unroll
                for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < Cfg::CB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, af[rb]), __builtin_bit_cast(f16x8, bf[cb]), acc[rb][cb], 0,
                            0, 0);
            }
        }
    }
}

// One BM x BN output tile over the k-tiles of split `split`.
template <class Cfg>
__device__ __forceinline__ void lp_tile(const TileProblem &P, int tm, int tn, int split, uint8_t *lds) {
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

    LpStage<Cfg> R;
    if (kt0 < kt1) {
        lp_load_tiles<Cfg>(P, m0, n0, kt0 * Cfg::BK, R);
        lp_store_tiles<Cfg>(lds, R);
    }
    __syncthreads();
    for (int kt = kt0; kt < kt1; ++kt) {
        const int cur = (kt - kt0) & 1;
        const bool more = kt + 1 < kt1;
        if (more) lp_load_tiles<Cfg>(P, m0, n0, (kt + 1) * Cfg::BK, R);
        lp_compute_stage<Cfg>(lds + cur * Cfg::STAGE, acc);
        if (more) lp_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, R);
        __syncthreads();
    }
    float *C;
    int64_t ldc;
    float scale;
    epilogue_target(P, split, C, ldc, scale);
    tile_epilogue<Cfg>(C, ldc, P.m, P.n, m0, n0, scale, acc);
}

template <int MODE, int BM, int BN, int BK>
__device__ __forceinline__ void LpCfg<MODE, BM, BN, BK>::run(const TileProblem &P, int tm, int tn, int split,
                                                         uint8_t *lds) {
    lp_tile<LpCfg<MODE, BM, BN, BK>>(P, tm, tn, split, lds);
}
