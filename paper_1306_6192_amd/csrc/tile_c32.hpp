// Complex-float output tile of C = A*B on gfx950 matrix cores
// (v_mfma_f32_32x32x2_f32).  The paper times the product for complex float
// matrices as well (Results section, Table 2's complex column).
//
// Operands are interleaved (re, im) float pairs; strides count complex
// elements.  Each complex multiply-add is four real ones on the matrix cores
// ("4M"): Re C += Re A Re B - Im A Im B, Im C += Re A Im B + Im A Re B, with
// the negation of Im A folded into the operand, so every real product is
// exact in float32 accumulation terms and no cancellation is introduced by
// the method itself (the 3-multiplication Gauss form is not used: its error
// bound is weaker).  The real and imaginary accumulators are separate
// 32x32 float32 blocks.
//
// Structure as in the FP32 tile: one workgroup of WM x WN waves owns a BM x BN
// complex tile and walks k in k-tiles of BK = 16 complex
// (128 bytes per row) through two LDS stages, one barrier per k-tile.
//
// MFMA operand layout (32x32x2, f32): lane l supplies A[l%32][kslot(l/32)]
// and B[kslot(l/32)][l%32]; the 32x32 result has, in lane l and register r,
// row 8*(r/4) + 4*(l/32) + r%4 and column l%32.  k order: within a chunk of
// 8 consecutive k, MFMA step t (0..3) consumes k = 8c + t in lanes 0..31 and
// k = 8c + 4 + t in lanes 32..63, so each lane reads its four complex A
// values of the chunk with one 32-byte LDS read.  Columns: lane l%32 = jj
// of a wave owning TN = 32*CB columns reads the CB consecutive complex B
// values at column CB*jj; block cb, lane column jj is output column
// CB*jj + cb, and the epilogue stores CB consecutive complex values per row.
#pragma once

#include "tile_common.hpp"

template <int BM_, int BN_, int WM_ = 2, int WN_ = 2>
struct C32Cfg {
    static constexpr int BM = BM_, BN = BN_, BK = 16;   // BK in complex elements
    static constexpr int WM = WM_, WN = WN_;          // waves along m and n
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int RB = TM / 32, CB = TN / 32;
    static constexpr int SA = 2 * BK + 4;   // LDS row stride of A (floats)
    static constexpr int SB = 2 * BN + 4;   // LDS row stride of B (floats)
    static constexpr int A_ELEMS = BM * SA, B_ELEMS = BK * SB;
    static constexpr int STAGE = A_ELEMS + B_ELEMS;
    static constexpr int LDS_BYTES = 2 * STAGE * 4;
    static constexpr int AV = BM * 2 * BK / 4 / THREADS;  // 16-byte loads per thread (A)
    static constexpr int BV = BK * 2 * BN / 4 / THREADS;  // 16-byte loads per thread (B)
    static_assert(RB >= 1 && (CB == 1 || CB == 2), "wave tile");
    static_assert(AV >= 1 && BV >= 1, "tile too small for the workgroup");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
    static constexpr int MFMA_K = 2;
    __device__ static void run(const TileProblem &P, int tm, int tn, int split, uint8_t *lds);
};

// Two consecutive complex values (four floats) of row r from complex column
// c, zero outside [0,R) x [0,Cn).
__device__ __forceinline__ f32x4 c32_load2(const float *__restrict__ P, int64_t ld, int r, int c, int R, int Cn) {
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r < R) {
        const float *p = P + 2 * ((int64_t)r * ld + c);
        if (c + 1 < Cn) {
            v = __builtin_bit_cast(f32x4, ld16(p));
        } else if (c < Cn) {
            const f32x2 h = __builtin_bit_cast(f32x2, *reinterpret_cast<const u32x2 *>(p));
            v[0] = h[0];
            v[1] = h[1];
        }
    }
    return v;
}

// CHECK = false: the whole blocks lie inside A and B (interior tiles).
template <class Cfg, bool CHECK = true>
__device__ __forceinline__ void c32_load_tiles(const TileProblem &P, int m0, int n0, int k0, f32x4 (&ra)[Cfg::AV],
                                               f32x4 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    const float *A = static_cast<const float *>(P.A);
    const float *B = static_cast<const float *>(P.B);
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 2);
        const int kv = (idx % (Cfg::BK / 2)) * 2;
        if constexpr (CHECK) ra[q] = c32_load2(A, P.lda, m0 + r, k0 + kv, P.m, P.k);
        else ra[q] = __builtin_bit_cast(f32x4, ld16(A + 2 * ((int64_t)(m0 + r) * P.lda + k0 + kv)));
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 2);
        const int cv = (idx % (Cfg::BN / 2)) * 2;
        if constexpr (CHECK) rb[q] = c32_load2(B, P.ldb, k0 + kr, n0 + cv, P.k, P.n);
        else rb[q] = __builtin_bit_cast(f32x4, ld16(B + 2 * ((int64_t)(k0 + kr) * P.ldb + n0 + cv)));
    }
}

template <class Cfg>
__device__ __forceinline__ void c32_store_tiles(float *stage, const f32x4 (&ra)[Cfg::AV],
                                                const f32x4 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    float *As = stage;
    float *Bs = stage + Cfg::A_ELEMS;
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 2);
        const int kv = (idx % (Cfg::BK / 2)) * 2;
        *reinterpret_cast<f32x4 *>(&As[r * Cfg::SA + 2 * kv]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 2);
        const int cv = (idx % (Cfg::BN / 2)) * 2;
        *reinterpret_cast<f32x4 *>(&Bs[kr * Cfg::SB + 2 * cv]) = rb[q];
    }
}

template <class Cfg>
__device__ __forceinline__ void c32_compute_stage(const float *stage, f32x16 (&re)[Cfg::RB][Cfg::CB],
                                                  f32x16 (&im)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const float *As = stage + (wm * Cfg::TM + l32) * Cfg::SA + 2 * (4 * g);
    const float *Bs = stage + Cfg::A_ELEMS + (4 * g) * Cfg::SB + 2 * (wn * Cfg::TN + Cfg::CB * l32);
#pragma unroll
    for (int kc = 0; kc < Cfg::BK / 8; ++kc) {
        f32x4 af[Cfg::RB][2];         // four complex A values: (re, im) x 4
        f32x4 bf[4];                  // CB complex B values per step (CB <= 2)
#pragma unroll
        for (int rb = 0; rb < Cfg::RB; ++rb) {
            const float *p = As + rb * 32 * Cfg::SA + 2 * (kc * 8);
            af[rb][0] = *reinterpret_cast<const f32x4 *>(p);
            af[rb][1] = *reinterpret_cast<const f32x4 *>(p + 4);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float *p = Bs + (kc * 8 + t) * Cfg::SB;
            if constexpr (Cfg::CB == 2) {
                bf[t] = *reinterpret_cast<const f32x4 *>(p);
            } else {
                const f32x2 h = *reinterpret_cast<const f32x2 *>(p);
                bf[t] = f32x4{h[0], h[1], 0.f, 0.f};
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb) {
                const float ar = af[rb][t >> 1][2 * (t & 1)];
                const float ai = af[rb][t >> 1][2 * (t & 1) + 1];
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb) {
                    const float br = bf[t][2 * cb], bi = bf[t][2 * cb + 1];
                    re[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, re[rb][cb], 0, 0, 0);
                    re[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, re[rb][cb], 0, 0, 0);
                    im[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, im[rb][cb], 0, 0, 0);
                    im[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, im[rb][cb], 0, 0, 0);
                }
            }
        }
    }
}

// Store the wave's complex accumulators to C: re(rb, cb, r) and im(rb, cb, r)
// give register r of the real and imaginary 32x32 blocks (rb, cb).
template <class Cfg, class Re, class Im>
__device__ __forceinline__ void c32_store(float *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0, Re re,
                                          Im im) {
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
            float v[2 * Cfg::CB];
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb) {
                v[2 * cb] = re(rb, cb, r);
                v[2 * cb + 1] = im(rb, cb, r);
            }
            float *p = C + 2 * ((int64_t)row * ldc + col);
            if (full_cols) {
                __builtin_memcpy(p, v, sizeof(v));
            } else {
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb)
                    if (col + cb < N) {
                        p[2 * cb] = v[2 * cb];
                        p[2 * cb + 1] = v[2 * cb + 1];
                    }
            }
        }
    }
}

template <class Cfg>
__device__ __forceinline__ void c32_epilogue(float *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0,
                                             const f32x16 (&re)[Cfg::RB][Cfg::CB],
                                             const f32x16 (&im)[Cfg::RB][Cfg::CB]) {
    c32_store<Cfg>(C, ldc, M, N, m0, n0, [&](int rb, int cb, int r) { return re[rb][cb][r]; },
                   [&](int rb, int cb, int r) { return im[rb][cb][r]; });
}

template <class Cfg>
__device__ __forceinline__ void c32_tile(const TileProblem &P, int tm, int tn, float *lds) {
    const int m0 = tm * Cfg::BM, n0 = tn * Cfg::BN;
    const int nkt = (P.k + Cfg::BK - 1) / Cfg::BK;

    f32x16 re[Cfg::RB][Cfg::CB], im[Cfg::RB][Cfg::CB];
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < Cfg::CB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                re[rb][cb][r] = 0.f;
                im[rb][cb][r] = 0.f;
            }

    f32x4 ra[Cfg::AV], rbv[Cfg::BV];
    if (nkt > 0) {
        c32_load_tiles<Cfg>(P, m0, n0, 0, ra, rbv);
        c32_store_tiles<Cfg>(lds, ra, rbv);
    }
    __syncthreads();
    // interior tiles: unmasked loads (same arithmetic as the masked loop)
    const bool interior = m0 + Cfg::BM <= P.m && n0 + Cfg::BN <= P.n && nkt * Cfg::BK <= P.k;
    if (interior) {
        for (int kt = 0; kt < nkt; ++kt) {
            const int cur = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) c32_load_tiles<Cfg, false>(P, m0, n0, (kt + 1) * Cfg::BK, ra, rbv);
            c32_compute_stage<Cfg>(lds + cur * Cfg::STAGE, re, im);
            if (more) c32_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, ra, rbv);
            __syncthreads();
        }
    } else {
        for (int kt = 0; kt < nkt; ++kt) {
            const int cur = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) c32_load_tiles<Cfg>(P, m0, n0, (kt + 1) * Cfg::BK, ra, rbv);
            c32_compute_stage<Cfg>(lds + cur * Cfg::STAGE, re, im);
            if (more) c32_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, ra, rbv);
            __syncthreads();
        }
    }
    c32_epilogue<Cfg>(P.C, P.ldc, P.m, P.n, m0, n0, re, im);
}

template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void C32Cfg<BM, BN, WM, WN>::run(const TileProblem &P, int tm, int tn, int,
                                                            uint8_t *lds) {
    c32_tile<C32Cfg<BM, BN, WM, WN>>(P, tm, tn, reinterpret_cast<float *>(lds));
}
