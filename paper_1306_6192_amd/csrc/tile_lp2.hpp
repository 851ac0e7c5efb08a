// Asynchronous-copy output tile (BF16, F16, FP8, FP32, binary64 and complex
// float).
//
// Same arithmetic as the register-staged tiles (tile_lp.hpp for BF16, F16
// and FP8, tile_f32.hpp for FP32, tile_f64.hpp for binary64, tile_c32.hpp
// for complex float: same MFMA instructions, same k order, so each pair
// produces identical bits), different data movement:
//   * A and B go from HBM straight into LDS with 16-byte direct loads
//     (global_load_lds_dwordx4): no staging registers and no register
//     transpose; lane L of one such load lands at LDS base + 16*L.
//   * A ring of STAGES LDS buffers keeps STAGES-1 k-tiles in flight while one
//     is consumed; each wave waits (vmcnt) only for its own oldest tile and one
//     barrier per k-tile publishes it.
//   * FP32 (v_mfma_f32_32x32x2_f32): one k-step is 8 consecutive k, read as
//     one 16-byte A chunk per lane (k = 8c + 4(l/32) .. + 3, as in
//     tile_f32.hpp) and, per MFMA t = 0..3, the CB consecutive floats of B row
//     8c + 4(l/32) + t at column CB*(l%32) of the wave's columns; B rows need
//     no swizzle (32 lanes read 32 consecutive 8- or 16-byte pieces).
//   * binary64 (v_mfma_f64_16x16x4_f64, 16x16 accumulator blocks): A rows of
//     a k-tile are 128 bytes (16 doubles, the register-staged tile's k-tile),
//     one step per k-tile: lane (l%16, g = l/16) reads doubles 4g .. 4g + 3
//     of its row as two 16-byte chunks, and MFMA t = 0..3 takes k = 4g + t;
//     B row 4g + t is read at the column pairs 32h + 2(l%16) of tile_f64.hpp.
//   * complex float (interleaved (re, im) pairs, four real 32x32x2 MFMAs per
//     complex term): A rows of a k-tile are 128 bytes (16 complex, the
//     register-staged tile's k-tile), two steps of 8 k; lane (l%32, g =
//     l/32) reads complex k = 8c + 4g .. + 3 of its row as two 16-byte
//     chunks and B row 8c + 4g + t at complex column CB*(l%32); the real and
//     imaginary parts of block cb accumulate in acc[rb][2cb] and
//     acc[rb][2cb + 1].
//   * 16- and 8-bit B stays row-major (k x n) in LDS; the MFMA B operand
//     (consecutive k of one column per lane) is gathered with the transposing
//     LDS reads
//     ds_read_b64_tr_b16 / ds_read_b64_tr_b8.  Within each group of 16 lanes,
//     lane j receives element j%4 (b16; j%8 for b8) of the 8-byte chunk
//     addressed by lane 4r + j/4 (b8: 2r + j/8), for r = 0..3 (b8: 0..7); so
//     lane 4r + c addressing B[k0+r][n0+4c..] yields B[k0..k0+3][n0+j] in
//     lane j (b8: lane 2r + c addressing B[k0+r][n0+8c..]).
//   * Rows are XOR-swizzled at 16-byte granularity so that the fragment reads
//     of 16 (A) or 4-8 (B) consecutive rows hit distinct LDS banks; the
//     swizzle is applied on the global side of the direct loads (each lane
//     picks which logical chunk it fetches), since the LDS side is fixed.
// Shape requirements of the 16-byte loads (checked on the host; other shapes
// use the register-staged tiles): k and n multiples of the 16-byte chunk
// (2 x 64-bit, 4 x 32-bit, 8 x 16-bit or 16 x 8-bit), row strides multiples
// of 16 bytes, 16-byte aligned A and B.  The FP32 tiles with 4-byte loads
// (one element per lane, global_load_lds_dword) take any shape.  Rows of A
// beyond m and columns of B beyond n read clamped (valid, finite) data whose
// results are never stored; k beyond the end reads zeros.
#pragma once

#include <type_traits>

#include "tile_c32.hpp"
#include "tile_common.hpp"
#include "tile_f64.hpp"

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef int i32x2 __attribute__((ext_vector_type(2)));

// A 16-byte chunk of zeros in device memory: the source of k positions past
// the end of the matrices.
static __device__ __attribute__((aligned(16))) uint32_t g_zero_chunk[4];

// s_waitcnt vmcnt(N) with the other counters left alone (gfx9 encoding:
// vmcnt[3:0] and [15:14], expcnt[6:4] = 7, lgkmcnt[11:8] = 15).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// AROWB_: bytes of an A row per k-tile (0: the mode's own, 64 or 128).
// LDB_: bytes each lane moves per direct load: 16 (global_load_lds_dwordx4;
// k, n, strides and bases in whole 16-byte chunks) or 4 (FP32 only,
// global_load_lds_dword: one element per lane, so any shape, stride and
// alignment; the LDS image is the same, so are the bits).
// MB_: accumulator block edge of the 16-bit tiles: 32 (v_mfma_f32_32x32x16,
// k-steps of 16) or 16 (v_mfma_f32_16x16x32, k-steps of 32; one such MFMA
// gives the bits of two 32x32x16 MFMAs over its two k halves, so both tile
// families of a mode give the same results).
template <int MODE_, int BM_, int BN_, int STAGES_, int WM_ = 2, int WN_ = 2, int AROWB_ = 0, int LDB_ = 16,
          int MB_ = 32>
struct Lp2Cfg {
    static constexpr int MODE = MODE_;
    static constexpr int BM = BM_, BN = BN_, STAGES = STAGES_;
    static constexpr int WM = WM_, WN = WN_;            // waves along m and n
    static constexpr int WAVES = WM * WN;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr bool F32 = (MODE == GEMM_MODE_F32);
    static constexpr bool F64 = (MODE == GEMM_MODE_F64);
    static constexpr bool C32 = (MODE == GEMM_MODE_C32);
    static constexpr bool H16 = (MODE == GEMM_MODE_BF16 || MODE == GEMM_MODE_F16);
    static_assert(MB_ == 32 || (MB_ == 16 && H16), "16x16 blocks for the 16-bit tiles only");
    static constexpr bool M16 = H16 && MB_ == 16;      // 16x16x32 MFMAs
    static constexpr int BLK = F64 ? 16 : MB_;          // accumulator block edge
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int RB = TM / BLK, CB = TN / BLK;
    static constexpr int CBA = C32 ? 2 * CB : CB;       // accumulator blocks per row block
    static constexpr int ESZ = (MODE == GEMM_MODE_F8E4M3) ? 1 : (F64 || C32) ? 8 : F32 ? 4 : 2;
    static constexpr int CE = 16 / ESZ;                 // elements per 16-byte chunk
    static constexpr int A_ROWB = AROWB_ ? AROWB_ : (F64 || C32) ? 128 : 64;   // bytes of an A row per k-tile
    static constexpr int A_CPR = A_ROWB / 16;           // 16-byte chunks per A row
    static constexpr int BK = A_ROWB / ESZ;             // k per k-tile
    // k per step: one MFMA (16- and 8-bit), four 32x32x2 MFMAs (FP32), four
    // 16x16x4 MFMAs (binary64), four times four 32x32x2 MFMAs (complex)
    static constexpr int KCH = (MODE == GEMM_MODE_F8E4M3) ? 64 : F64 ? 16 : (F32 || C32) ? 8 : M16 ? 32 : 16;
    static constexpr int MFMA_K = (F32 || C32) ? 2 : F64 ? 4 : KCH;
    static constexpr int STEPS = BK / KCH;
    static constexpr bool FOUR = F32 || F64 || C32;     // four k-slots per block per step
    static constexpr int NPB = FOUR ? 4 : CB;           // B fragment reads per step
    static constexpr int NP = RB + NPB;                 // fragment reads per step
    static constexpr int NM = RB * CB * (FOUR ? 4 : 1) * (C32 ? 4 : 1);   // MFMAs per step
    typedef typename std::conditional<F64, f64x4, typename std::conditional<M16, f32x4, f32x16>::type>::type Acc;
    static constexpr int B_ROWB = BN * ESZ;
    static constexpr int B_CPR = B_ROWB / 16;           // 16-byte chunks per B row
    static constexpr int A_STAGE = BM * A_ROWB;
    static constexpr int B_STAGE = BK * B_ROWB;
    static constexpr int STAGE = A_STAGE + B_STAGE;
    static constexpr int LDS_BYTES = STAGES * STAGE;
    static constexpr int LDB = LDB_;                    // bytes per lane per direct load
    static constexpr int WLOAD = 64 * LDB;              // bytes one wave moves per direct load
    static_assert(LDB == 16 || (LDB == 4 && F32), "16-byte loads, or 4-byte loads of float32 elements");
    static constexpr int A_LOADS = A_STAGE / WLOAD / WAVES;  // direct loads per wave per k-tile
    static constexpr int B_LOADS = B_STAGE / WLOAD / WAVES;
    static constexpr int LOADS = A_LOADS + B_LOADS;
    static_assert(RB >= 1 && CB >= 1, "wave tile");
    static_assert(A_LOADS >= 1 && B_LOADS >= 1 && A_LOADS * WLOAD * WAVES == A_STAGE &&
                      B_LOADS * WLOAD * WAVES == B_STAGE,
                  "stage sizes must be whole numbers of one load per wave");
    static_assert(STAGES >= 2 && (STAGES - 1) * LOADS < 64, "vmcnt range");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
    // physical chunk of logical chunk c in A row r / B row k
    // 64-byte A rows (4 chunks): a fragment read of 16 consecutive rows (one
    // 16-lane phase of a 16-byte LDS read on the 64 banks) touches 4 rows of
    // each (r mod 4) class: XOR-ing the chunk with bits 1-2 of the row gives
    // those 16 rows distinct banks (and 8 consecutive rows too).  128-byte
    // rows (8 chunks): 16 rows hold 2 of each (r mod 2) class, and bits 1-3
    // of the row spread each class over 8 chunks.
    __device__ static __forceinline__ int a_swz(int r) {
        if constexpr (A_CPR == 8) return (r >> 1) & 7;
        return ((r >> 1) ^ (r >> 2)) & 3;
    }
    __device__ static __forceinline__ int b_swz(int k) {
        if constexpr (F32 || F64 || C32) return 0;
        return (ESZ == 2 ? 4 * (k & 3) : 2 * (k & 7)) & (B_CPR - 1);
    }
    __device__ static void run(const TileProblem &P, int tm, int tn, int split, uint8_t *lds);
};

// One 16-byte direct load per lane into LDS at `lds` + 16 * lane.  Written as
// inline assembly (M0 = LDS address) so that the compiler does not treat the
// transfer as an LDS write it must wait for before every later LDS read: the
// pipeline waits for it explicitly (wait_vmcnt before the k-tile's barrier).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void load_lds16(const void *src, uint32_t dst) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(dst), "v"(src) : "memory", "m0");
}

// The same with 4 bytes per lane: lane L lands at `dst` + 4 * L.
__device__ __forceinline__ void load_lds4(const void *src, uint32_t dst) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, off" ::"s"(dst), "v"(src) : "memory", "m0");
}

// LDS byte address of a pointer into the workgroup's shared array, made
// wave-uniform (one conversion per tile, not per load).
__device__ __forceinline__ uint32_t lds_addr(const uint8_t *p) {
    const uint32_t a = (uint32_t)(uintptr_t)((const __attribute__((address_space(3))) uint8_t *)p);
    return __builtin_amdgcn_readfirstlane(a);
}
#pragma clang diagnostic pop

// Per-lane sources of this wave's direct loads, computed once per output
// tile: the k-tile starting at k0 then only adds k0 times the k stride.
template <class Cfg>
struct Lp2Src {
    const uint8_t *a[Cfg::A_LOADS];   // A row start + logical chunk (element)
    int ak[Cfg::A_LOADS];             // k of that chunk (element) within a k-tile
    const uint8_t *b[Cfg::B_LOADS];   // B row kr of the k-tile + column chunk (element)
    int bk[Cfg::B_LOADS];             // kr
    int64_t bstep;                    // bytes between consecutive B rows
    int kend;                         // loads at k >= kend read the zero chunk
    uint32_t dst_a, dst_b;            // this wave's first A / B destination in stage 0
};

template <class Cfg>
__device__ __forceinline__ void lp2_sources(const TileProblem &P, int m0, int n0, int kend, const uint8_t *lds,
                                            Lp2Src<Cfg> &S) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *A = static_cast<const uint8_t *>(P.A);
    const uint8_t *B = static_cast<const uint8_t *>(P.B);
    if constexpr (Cfg::LDB == 16) {
#pragma unroll
        for (int j = 0; j < Cfg::A_LOADS; ++j) {
            const int t = wave * Cfg::A_LOADS + j;          // 1 KiB piece of the A stage
            const int r = (64 / Cfg::A_CPR) * t + lane / Cfg::A_CPR;   // tile row
            const int c = (lane % Cfg::A_CPR) ^ Cfg::a_swz(r);           // logical chunk at physical chunk lane % A_CPR
            const int row = min(m0 + r, P.m - 1);
            S.ak[j] = c * Cfg::CE;
            S.a[j] = A + ((int64_t)row * P.lda + S.ak[j]) * Cfg::ESZ;
        }
#pragma unroll
        for (int j = 0; j < Cfg::B_LOADS; ++j) {
            const int slot = 64 * (wave * Cfg::B_LOADS + j) + lane;
            const int kr = slot / Cfg::B_CPR;
            const int c = (slot % Cfg::B_CPR) ^ Cfg::b_swz(kr);
            const int n = min(n0 + c * Cfg::CE, P.n - Cfg::CE);
            S.bk[j] = kr;
            S.b[j] = B + ((int64_t)kr * P.ldb + n) * Cfg::ESZ;
        }
    } else {
        // 4-byte loads: lane L of load j writes stage byte WLOAD * (the wave's
        // piece j) + 4 L, i.e. one element of a row's physical 16-byte chunk;
        // it fetches that element of the logical chunk the swizzle puts there
#pragma unroll
        for (int j = 0; j < Cfg::A_LOADS; ++j) {
            const int byte = Cfg::WLOAD * (wave * Cfg::A_LOADS + j) + Cfg::LDB * lane;
            const int r = byte / Cfg::A_ROWB;                                   // tile row
            const int o = byte % Cfg::A_ROWB;
            const int c = (o / 16) ^ Cfg::a_swz(r);                             // logical chunk
            const int row = min(m0 + r, P.m - 1);
            S.ak[j] = c * Cfg::CE + (o % 16) / Cfg::ESZ;
            S.a[j] = A + ((int64_t)row * P.lda + S.ak[j]) * Cfg::ESZ;
        }
#pragma unroll
        for (int j = 0; j < Cfg::B_LOADS; ++j) {
            const int byte = Cfg::WLOAD * (wave * Cfg::B_LOADS + j) + Cfg::LDB * lane;
            const int kr = byte / Cfg::B_ROWB;
            const int o = byte % Cfg::B_ROWB;
            const int c = (o / 16) ^ Cfg::b_swz(kr);
            // columns past n: a valid element whose products are never stored
            const int n = min(n0 + c * Cfg::CE + (o % 16) / Cfg::ESZ, P.n - 1);
            S.bk[j] = kr;
            S.b[j] = B + ((int64_t)kr * P.ldb + n) * Cfg::ESZ;
        }
    }
    S.bstep = P.ldb * Cfg::ESZ;
    S.kend = kend;
    const uint32_t base = lds_addr(lds);
    S.dst_a = base + Cfg::WLOAD * (wave * Cfg::A_LOADS);
    S.dst_b = base + Cfg::A_STAGE + Cfg::WLOAD * (wave * Cfg::B_LOADS);
}

// Issue direct load j (A loads first, then B) of this wave for the k-tile
// starting at k0 into the stage at LDS byte offset `soff`.  CHECK: chunks at
// k >= kend read the zero chunk; without it the caller guarantees that the
// whole k-tile lies before kend.
template <class Cfg, bool CHECK>
__device__ __forceinline__ void lp2_issue_one(const Lp2Src<Cfg> &S, int k0, uint32_t soff, int j) {
    if (j < Cfg::A_LOADS) {
        const void *src = (!CHECK || k0 + S.ak[j] < S.kend) ? (const void *)(S.a[j] + (int64_t)k0 * Cfg::ESZ)
                                                             : (const void *)g_zero_chunk;
        if constexpr (Cfg::LDB == 16) load_lds16(src, S.dst_a + soff + Cfg::WLOAD * j);
        else load_lds4(src, S.dst_a + soff + Cfg::WLOAD * j);
    } else {
        const int b = j - Cfg::A_LOADS;
        const void *src = (!CHECK || k0 + S.bk[b] < S.kend) ? (const void *)(S.b[b] + (int64_t)k0 * S.bstep)
                                                             : (const void *)g_zero_chunk;
        if constexpr (Cfg::LDB == 16) load_lds16(src, S.dst_b + soff + Cfg::WLOAD * b);
        else load_lds4(src, S.dst_b + soff + Cfg::WLOAD * b);
    }
}

template <class Cfg, bool CHECK = true>
__device__ __forceinline__ void lp2_issue(const Lp2Src<Cfg> &S, int k0, uint32_t soff) {
#pragma unroll
    for (int j = 0; j < Cfg::LOADS; ++j) lp2_issue_one<Cfg, CHECK>(S, k0, soff, j);
}

// MFMA operand fragments of one k-step (KCH consecutive k) for the wave's
// RB x CB accumulator blocks.  Kind 0: 16-bit, 1: FP8, 2: FP32, 3: binary64,
// 4: complex float (for the last three, b[t] holds the CB values of MFMA
// slot t, one per accumulator block column; binary64 and complex a[rb] hold
// the lane's four k as two 16-byte chunks).
template <int CB> struct Lp2FVec;
template <> struct Lp2FVec<1> { typedef float T; };
template <> struct Lp2FVec<2> { typedef f32x2 T; };
template <> struct Lp2FVec<4> { typedef f32x4 T; };

template <class Cfg,
          int KIND = (Cfg::MODE == GEMM_MODE_F8E4M3) ? 1 : Cfg::F32 ? 2 : Cfg::F64 ? 3 : Cfg::C32 ? 4 : 0>
struct Lp2Frag;
template <class Cfg>
struct Lp2Frag<Cfg, 0> {
    u32x4 a[Cfg::RB];
    u32x4 b[Cfg::CB];
};
template <class Cfg>
struct Lp2Frag<Cfg, 1> {
    i32x8 a[Cfg::RB];
    i32x8 b[Cfg::CB];
};
template <class Cfg>
struct Lp2Frag<Cfg, 2> {
    f32x4 a[Cfg::RB];
    typename Lp2FVec<Cfg::CB>::T b[4];
};
template <class Cfg>
struct Lp2Frag<Cfg, 3> {
    f64x2 a[Cfg::RB][2];
    typename DVec<Cfg::CB>::T b[4];
};
template <class Cfg>
struct Lp2Frag<Cfg, 4> {
    f32x4 a[Cfg::RB][2];                        // four complex k: (re, im) x 2, twice
    typename Lp2FVec<2 * Cfg::CB>::T b[4];      // CB complex values of MFMA slot t
};

// Read piece p of the fragments of k-step kc of the k-tile held in `stage`:
// p < RB is A row block p, otherwise B column block p - RB (FP32: the B
// values of MFMA p - RB for all CB column blocks).
template <class Cfg>
__device__ __forceinline__ void lp2_read_piece(const uint8_t *stage, int kc, int p, Lp2Frag<Cfg> &F) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const int p16 = lane & 15, G = lane >> 4;
    const uint8_t *As = stage;
    const uint8_t *Bs = stage + Cfg::A_STAGE;
    if constexpr (Cfg::C32) {
        if (p < Cfg::RB) {
            const int r = wm * Cfg::TM + p * 32 + l32;
            const uint8_t *row = As + r * Cfg::A_ROWB;
            F.a[p][0] = *reinterpret_cast<const f32x4 *>(row + 16 * ((4 * kc + 2 * g) ^ Cfg::a_swz(r)));
            F.a[p][1] = *reinterpret_cast<const f32x4 *>(row + 16 * ((4 * kc + 2 * g + 1) ^ Cfg::a_swz(r)));
        } else {
            const int t = p - Cfg::RB;
            const float *row = reinterpret_cast<const float *>(Bs + (8 * kc + 4 * g + t) * Cfg::B_ROWB);
            F.b[t] = *reinterpret_cast<const typename Lp2FVec<2 * Cfg::CB>::T *>(
                row + 2 * (wn * Cfg::TN + Cfg::CB * l32));
        }
    } else if constexpr (Cfg::F64) {
        const int l16 = lane & 15, g4 = lane >> 4;
        if (p < Cfg::RB) {
            const int r = wm * Cfg::TM + p * 16 + l16;
            const uint8_t *row = As + r * Cfg::A_ROWB;
            F.a[p][0] = *reinterpret_cast<const f64x2 *>(row + 16 * ((2 * g4) ^ Cfg::a_swz(r)));
            F.a[p][1] = *reinterpret_cast<const f64x2 *>(row + 16 * ((2 * g4 + 1) ^ Cfg::a_swz(r)));
        } else {
            const int t = p - Cfg::RB;
            const double *row = reinterpret_cast<const double *>(Bs + (4 * g4 + t) * Cfg::B_ROWB) + wn * Cfg::TN;
            if constexpr (Cfg::CB == 4) {
                const f64x2 lo = *reinterpret_cast<const f64x2 *>(row + 2 * l16);
                const f64x2 hi = *reinterpret_cast<const f64x2 *>(row + 32 + 2 * l16);
                F.b[t] = f64x4{lo[0], lo[1], hi[0], hi[1]};
            } else if constexpr (Cfg::CB == 2) {
                F.b[t] = *reinterpret_cast<const f64x2 *>(row + 2 * l16);
            } else {
                F.b[t] = row[l16];
            }
        }
    } else if constexpr (Cfg::F32) {
        if (p < Cfg::RB) {
            const int r = wm * Cfg::TM + p * 32 + l32;
            F.a[p] = *reinterpret_cast<const f32x4 *>(As + r * Cfg::A_ROWB + 16 * ((2 * kc + g) ^ Cfg::a_swz(r)));
        } else {
            const int t = p - Cfg::RB;
            const int k = 8 * kc + 4 * g + t;
            const float *row = reinterpret_cast<const float *>(Bs + k * Cfg::B_ROWB);
            F.b[t] = *reinterpret_cast<const typename Lp2FVec<Cfg::CB>::T *>(row + wn * Cfg::TN + Cfg::CB * l32);
        }
    } else if constexpr (Cfg::MODE == GEMM_MODE_F8E4M3) {
        if (p < Cfg::RB) {
            const int rb = p;
            const int r = wm * Cfg::TM + rb * 32 + l32;
            const uint8_t *row = As + r * Cfg::A_ROWB;
            // step kc covers chunks 4 kc .. 4 kc + 3 of the row (64 k; one
            // step per k-tile with 64-byte rows, two with 128-byte rows)
            const u32x4 lo = *reinterpret_cast<const u32x4 *>(row + 16 * ((4 * kc + 2 * g) ^ Cfg::a_swz(r)));
            const u32x4 hi = *reinterpret_cast<const u32x4 *>(row + 16 * ((4 * kc + 2 * g + 1) ^ Cfg::a_swz(r)));
            F.a[rb] = (i32x8){(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3],
                              (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
        } else {
            const int cb = p - Cfg::RB;
            const int n = wn * Cfg::TN + cb * 32 + 16 * (G & 1) + 8 * (p16 & 1);
            i32x2 q[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int k = 64 * kc + 32 * (G >> 1) + 8 * h + (p16 >> 1);
                const uint8_t *a = Bs + k * Cfg::B_ROWB + 16 * ((n >> 4) ^ Cfg::b_swz(k)) + (n & 15);
                q[h] = __builtin_amdgcn_ds_read_tr8_b64_v2i32((__attribute__((address_space(3))) i32x2 *)a);
            }
            F.b[cb] = (i32x8){q[0][0], q[0][1], q[1][0], q[1][1], q[2][0], q[2][1], q[3][0], q[3][1]};
        }
    } else if constexpr (Cfg::M16) {
        // 16x16x32: lane (l%16, G = l/16) holds k = 8G .. 8G + 7 of row l%16
        // (A) and of column l%16 (B) of the step's 32 k
        if (p < Cfg::RB) {
            const int rb = p;
            const int r = wm * Cfg::TM + rb * 16 + p16;
            F.a[rb] = *reinterpret_cast<const u32x4 *>(As + r * Cfg::A_ROWB + 16 * ((4 * kc + G) ^ Cfg::a_swz(r)));
        } else {
            const int cb = p - Cfg::RB;
            const int n = wn * Cfg::TN + cb * 16 + 4 * (p16 & 3);
            s16x4 hv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 32 * kc + 8 * G + 4 * h + (p16 >> 2);
                const uint8_t *a = Bs + k * Cfg::B_ROWB + 16 * ((n >> 3) ^ Cfg::b_swz(k)) + 2 * (n & 7);
                hv[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)a);
            }
            const i32x2 lo = __builtin_bit_cast(i32x2, hv[0]);
            const i32x2 hi = __builtin_bit_cast(i32x2, hv[1]);
            F.b[cb] = (u32x4){(uint32_t)lo[0], (uint32_t)lo[1], (uint32_t)hi[0], (uint32_t)hi[1]};
        }
    } else {
        if (p < Cfg::RB) {
            const int rb = p;
            const int r = wm * Cfg::TM + rb * 32 + l32;
            F.a[rb] = *reinterpret_cast<const u32x4 *>(As + r * Cfg::A_ROWB + 16 * ((2 * kc + g) ^ Cfg::a_swz(r)));
        } else {
            const int cb = p - Cfg::RB;
            const int n = wn * Cfg::TN + cb * 32 + 16 * (G & 1) + 4 * (p16 & 3);
            s16x4 hv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 16 * kc + 8 * (G >> 1) + 4 * h + (p16 >> 2);
                const uint8_t *a = Bs + k * Cfg::B_ROWB + 16 * ((n >> 3) ^ Cfg::b_swz(k)) + 2 * (n & 7);
                hv[h] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)a);
            }
            const i32x2 lo = __builtin_bit_cast(i32x2, hv[0]);
            const i32x2 hi = __builtin_bit_cast(i32x2, hv[1]);
            F.b[cb] = (u32x4){(uint32_t)lo[0], (uint32_t)lo[1], (uint32_t)hi[0], (uint32_t)hi[1]};
        }
    }
}

template <class Cfg>
__device__ __forceinline__ void lp2_read(const uint8_t *stage, int kc, Lp2Frag<Cfg> &F) {
#pragma unroll
    for (int p = 0; p < Cfg::NP; ++p) lp2_read_piece<Cfg>(stage, kc, p, F);
}

// MFMA i (0 .. NM-1) of one k-step.  16- and 8-bit: the one MFMA of
// accumulator block (i / CB, i % CB).  FP32 and binary64: MFMA t = i / (RB CB)
// of block ((i / CB) % RB, i % CB), so that consecutive MFMAs feed different
// accumulators and each block sums t = 0, 1, 2, 3 in order.
template <class Cfg>
__device__ __forceinline__ void lp2_mfma1(const Lp2Frag<Cfg> &F, typename Cfg::Acc (&acc)[Cfg::RB][Cfg::CBA], int i) {
    if constexpr (Cfg::C32) {
        // slot t, then product j = 0..3 (Re += ar br, Re += (-ai) bi,
        // Im += ar bi, Im += ai br), then the blocks: each accumulator still
        // receives its products in the register-staged tile's order
        constexpr int NB = Cfg::RB * Cfg::CB;
        const int t = i / (4 * NB), j = (i / NB) % 4, rb = (i / Cfg::CB) % Cfg::RB, cb = i % Cfg::CB;
        const float ar = F.a[rb][t >> 1][2 * (t & 1)], ai = F.a[rb][t >> 1][2 * (t & 1) + 1];
        float br, bi;
        if constexpr (Cfg::CB == 1) {
            br = F.b[t][0];
            bi = F.b[t][1];
        } else {
            br = F.b[t][2 * cb];
            bi = F.b[t][2 * cb + 1];
        }
        if (j == 0) acc[rb][2 * cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc[rb][2 * cb], 0, 0, 0);
        else if (j == 1) acc[rb][2 * cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, acc[rb][2 * cb], 0, 0, 0);
        else if (j == 2) acc[rb][2 * cb + 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, acc[rb][2 * cb + 1], 0, 0, 0);
        else acc[rb][2 * cb + 1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, acc[rb][2 * cb + 1], 0, 0, 0);
    } else if constexpr (Cfg::F64) {
        const int t = i / (Cfg::RB * Cfg::CB), rb = (i / Cfg::CB) % Cfg::RB, cb = i % Cfg::CB;
        double bv;
        if constexpr (Cfg::CB == 1) bv = F.b[t];
        else bv = F.b[t][cb];
        acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(F.a[rb][t >> 1][t & 1], bv, acc[rb][cb], 0, 0, 0);
    } else if constexpr (Cfg::F32) {
        const int t = i / (Cfg::RB * Cfg::CB), rb = (i / Cfg::CB) % Cfg::RB, cb = i % Cfg::CB;
        float bv;
        if constexpr (Cfg::CB == 1) bv = F.b[t];
        else bv = F.b[t][cb];
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(F.a[rb][t], bv, acc[rb][cb], 0, 0, 0);
    } else {
        const int rb = i / Cfg::CB, cb = i % Cfg::CB;
        if constexpr (Cfg::MODE == GEMM_MODE_F8E4M3)
            acc[rb][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(F.a[rb], F.b[cb], acc[rb][cb], 0, 0, 0,
                                                                         0, 0, 0);
        else if constexpr (Cfg::M16 && Cfg::MODE == GEMM_MODE_BF16)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, F.a[rb]), __builtin_bit_cast(bf16x8, F.b[cb]), acc[rb][cb], 0, 0, 0);
        else if constexpr (Cfg::M16)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(f16x8, F.a[rb]), __builtin_bit_cast(f16x8, F.b[cb]), acc[rb][cb], 0, 0, 0);
        else if constexpr (Cfg::MODE == GEMM_MODE_BF16)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, F.a[rb]), __builtin_bit_cast(bf16x8, F.b[cb]), acc[rb][cb], 0, 0, 0);
        else
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, F.a[rb]), __builtin_bit_cast(f16x8, F.b[cb]), acc[rb][cb], 0, 0, 0);
    }
}

// Epilogue of the 16x16 blocks: lane l, register i of block (rb, cb) holds
// row 16 rb + 4 (l/16) + i, column 16 cb + l%16 of the wave's tile.
template <class Cfg>
__device__ __forceinline__ void lp2_epilogue16(float *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0,
                                               float scale, const f32x4 (&acc)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int p16 = lane & 15, G = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + wm * Cfg::TM + rb * 16 + 4 * G + i;
            if (row >= M) continue;
            float *p = C + (int64_t)row * ldc;
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb) {
                const int col = n0 + wn * Cfg::TN + cb * 16 + p16;
                if (col < N) p[col] = acc[rb][cb][i] * scale;
            }
        }
}

// Natural-column epilogue: lane l%32 of accumulator block cb holds output
// column 32*cb + l%32 of the wave's columns.
template <class Cfg>
__device__ __forceinline__ void lp2_epilogue(float *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0,
                                             float scale, const f32x16 (&acc)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = m0 + wm * Cfg::TM + rb * 32 + 8 * (r >> 2) + 4 * g + (r & 3);
            if (row >= M) continue;
            float *p = C + (int64_t)row * ldc;
#pragma unroll
            for (int cb = 0; cb < Cfg::CB; ++cb) {
                const int col = n0 + wn * Cfg::TN + cb * 32 + l32;
                if (col < N) p[col] = acc[rb][cb][r] * scale;
            }
        }
}

// One k-step of the software pipeline, in one of two fixed forms so that the
// loop body has no data-dependent branches:
//   * inner step (the next step reads the same k-tile): this step's MFMAs,
//     each followed by one piece of the next step's fragment reads;
//   * boundary step (the next step starts a new k-tile): the first half of
//     the MFMAs, retire this wave's LDS reads, wait for this wave's loads of
//     the next k-tile, synchronise the workgroup (which publishes that k-tile
//     and frees the stage just consumed), then the other half of the MFMAs
//     interleaved with the reads of the next k-tile's first fragments and
//     the refill of the freed stage with the k-tile STAGES ahead.
// Scheduling barriers pin this interleaving: the matrix cores then always
// have an MFMA queued while the wave issues its reads and loads, and the
// compiler cannot sink MFMAs below the workgroup barrier (they touch no
// memory) or pile the reads up in front of the boundary's LDS wait.
// `i` is the k-tile and `u` = i mod STAGES its stage; the callers unroll over
// u, so every LDS address is a constant offset from a few base registers.
// Loads are issued for k-tiles past the end too (their sources are the zero
// chunk), which keeps the number of loads in flight, and so every wait, the
// same in every iteration.  CHECK selects the k-bounded form of the loads.
template <class Cfg, bool BOUNDARY, bool CHECK>
__device__ __forceinline__ void lp2_step(const Lp2Src<Cfg> &S, int kt0, int i, int u, int kc, uint8_t *lds,
                                         const Lp2Frag<Cfg> &cur, Lp2Frag<Cfg> &nxt,
                                         typename Cfg::Acc (&acc)[Cfg::RB][Cfg::CBA]) {
    constexpr int NP = Cfg::NP;                     // fragment pieces per step
    constexpr int NM = Cfg::NM;                     // MFMAs per step
    if constexpr (BOUNDARY) {
        // MFMAs before the barrier
        constexpr int H = Cfg::FOUR ? NM / 2 : ((Cfg::RB + 1) / 2) * Cfg::CB;
        constexpr int W = NP + Cfg::LOADS;                 // work items after it
        constexpr int PER = (W + (NM - H) - 1) / (NM - H);
        static_assert(H < NM && (NM - H) * PER >= W, "every read and refill load is issued");
#pragma unroll
        for (int t = 0; t < H; ++t) lp2_mfma1<Cfg>(cur, acc, t);
        __builtin_amdgcn_sched_barrier(0);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        wait_vmcnt<(Cfg::STAGES - 2) * Cfg::LOADS>();
        __syncthreads();
        const uint8_t *next = lds + ((u + 1) % Cfg::STAGES) * Cfg::STAGE;
        const int k0 = (kt0 + i + Cfg::STAGES) * Cfg::BK;
#pragma unroll
        for (int t = H; t < NM; ++t) {
            lp2_mfma1<Cfg>(cur, acc, t);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int w = (t - H) * PER; w < (t - H + 1) * PER && w < W; ++w) {
                if (w < NP) lp2_read_piece<Cfg>(next, 0, w, nxt);
                else lp2_issue_one<Cfg, CHECK>(S, k0, u * Cfg::STAGE, w - NP);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const uint8_t *here = lds + u * Cfg::STAGE;
        // the NP reads of the next step go after the MFMAs, PER at a time:
        // after every other MFMA where a step has at least twice as many
        // MFMAs as reads (the FP32, binary64 and complex tiles), otherwise
        // after every MFMA
        constexpr int SPREAD = (Cfg::FOUR && NM >= 2 * NP) ? 2 : 1;
        constexpr int PER = (NP + NM / SPREAD - 1) / (NM / SPREAD);
        static_assert((NM / SPREAD) * PER >= NP, "every fragment piece of the next step is read");
#pragma unroll
        for (int t = 0; t < NM; ++t) {
            lp2_mfma1<Cfg>(cur, acc, t);
            __builtin_amdgcn_sched_barrier(0);
            if (t % SPREAD == 0) {
#pragma unroll
                for (int w = (t / SPREAD) * PER; w < (t / SPREAD + 1) * PER && w < NP; ++w)
                    lp2_read_piece<Cfg>(here, kc + 1, w, nxt);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// All steps of k-tile i (stage u).  On entry `fa` holds the tile's step-0
// fragments; on exit the next tile's step-0 fragments are in `fa` (an even
// number of steps per k-tile) or in `fb` (one step).
template <class Cfg, bool CHECK>
__device__ __forceinline__ void lp2_ktile(const Lp2Src<Cfg> &S, int kt0, int i, int u, uint8_t *lds,
                                          Lp2Frag<Cfg> &fa, Lp2Frag<Cfg> &fb, typename Cfg::Acc (&acc)[Cfg::RB][Cfg::CBA]) {
    if constexpr (Cfg::STEPS == 1) {
        lp2_step<Cfg, true, CHECK>(S, kt0, i, u, 0, lds, fa, fb, acc);
    } else {
#pragma unroll
        for (int kc = 0; kc + 2 < Cfg::STEPS; kc += 2) {
            lp2_step<Cfg, false, CHECK>(S, kt0, i, u, kc, lds, fa, fb, acc);
            lp2_step<Cfg, false, CHECK>(S, kt0, i, u, kc + 1, lds, fb, fa, acc);
        }
        lp2_step<Cfg, false, CHECK>(S, kt0, i, u, Cfg::STEPS - 2, lds, fa, fb, acc);
        lp2_step<Cfg, true, CHECK>(S, kt0, i, u, Cfg::STEPS - 1, lds, fb, fa, acc);
    }
}

// Two consecutive k-tiles i, i+1 in stages u, u+1 (u even), keeping the
// fragments in f0 at entry and exit.
template <class Cfg, bool CHECK>
__device__ __forceinline__ void lp2_pair(const Lp2Src<Cfg> &S, int kt0, int i, int u, int nt, bool guard,
                                         uint8_t *lds, Lp2Frag<Cfg> &f0, Lp2Frag<Cfg> &f1,
                                         typename Cfg::Acc (&acc)[Cfg::RB][Cfg::CBA]) {
    if (!guard || i < nt) lp2_ktile<Cfg, CHECK>(S, kt0, i, u, lds, f0, f1, acc);
    if (!guard || i + 1 < nt) {
        if constexpr (Cfg::STEPS % 2 == 0) lp2_ktile<Cfg, CHECK>(S, kt0, i + 1, u + 1, lds, f0, f1, acc);
        else lp2_ktile<Cfg, CHECK>(S, kt0, i + 1, u + 1, lds, f1, f0, acc);
    }
}

template <class Cfg>
__device__ __forceinline__ void lp2_tile(const TileProblem &P, int tm, int tn, int split, uint8_t *lds) {
    static_assert(Cfg::STEPS == 1 || Cfg::STEPS % 2 == 0, "pipeline written for 1 or an even number of steps per k-tile");
    static_assert(Cfg::STAGES % 2 == 0, "k-tiles are processed in pairs of stages");
    const int m0 = tm * Cfg::BM, n0 = tn * Cfg::BN;
    const int nkt = (P.k + Cfg::BK - 1) / Cfg::BK;
    const int kt0 = split * P.kt_per_split;
    const int kt1 = min(kt0 + P.kt_per_split, nkt);
    const int nt = max(0, kt1 - kt0);

    typename Cfg::Acc acc[Cfg::RB][Cfg::CBA];
    constexpr int NACC = sizeof(typename Cfg::Acc) / (Cfg::F64 ? 8 : 4);
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < Cfg::CBA; ++cb)
#pragma unroll
            for (int r = 0; r < NACC; ++r) acc[rb][cb][r] = 0;

    if (nt > 0) {
        // Fill the ring with k-tiles 0 .. STAGES-1 (those past kt1 read the
        // zero chunk; they are never used).
        Lp2Src<Cfg> S;
        const int kend = min(P.k, kt1 * Cfg::BK);
        lp2_sources<Cfg>(P, m0, n0, kend, lds, S);
        // k-tiles [0, nfull) of this split lie wholly before kend
        const int nfull = (kend - kt0 * Cfg::BK) / Cfg::BK;
#pragma unroll
        for (int s = 0; s < Cfg::STAGES; ++s) lp2_issue<Cfg>(S, (kt0 + s) * Cfg::BK, s * Cfg::STAGE);
        wait_vmcnt<(Cfg::STAGES - 1) * Cfg::LOADS>();
        __syncthreads();
        Lp2Frag<Cfg> f0, f1;
        lp2_read<Cfg>(lds, 0, f0);
        int i = 0;
        // rounds whose refills (k-tiles i + STAGES .. i + 2 STAGES - 1) are
        // whole: no k bound on the loads
        // (the stage loops are written out here: behind a helper function
        // the compiler unrolls them less and the eight-wave FP32 tiles spill)
        for (; i + 2 * Cfg::STAGES <= nfull; i += Cfg::STAGES) {
#pragma unroll
            for (int u = 0; u < Cfg::STAGES; u += 2)
                lp2_pair<Cfg, false>(S, kt0, i + u, u, nt, false, lds, f0, f1, acc);
        }
        for (; i + Cfg::STAGES <= nt; i += Cfg::STAGES) {
#pragma unroll
            for (int u = 0; u < Cfg::STAGES; u += 2)
                lp2_pair<Cfg, true>(S, kt0, i + u, u, nt, false, lds, f0, f1, acc);
        }
        // the last nt mod STAGES k-tiles (stages 0 ..)
#pragma unroll
        for (int u = 0; u < Cfg::STAGES; u += 2) lp2_pair<Cfg, true>(S, kt0, i + u, u, nt, true, lds, f0, f1, acc);
        wait_vmcnt<0>();   // the loads past the end have landed before the ring is reused
    }
    __syncthreads();       // the LDS ring may be refilled by this workgroup's next tile
    if constexpr (Cfg::F64) {
        // binary64 products have no split-K; P.C holds double elements
        f64_epilogue<Cfg>(reinterpret_cast<double *>(P.C), P.ldc, P.m, P.n, m0, n0, acc);
    } else if constexpr (Cfg::C32) {
        // nor do complex ones; P.C holds interleaved complex elements
        c32_store<Cfg>(P.C, P.ldc, P.m, P.n, m0, n0, [&](int rb, int cb, int r) { return acc[rb][2 * cb][r]; },
                       [&](int rb, int cb, int r) { return acc[rb][2 * cb + 1][r]; });
    } else {
        float *C;
        int64_t ldc;
        float scale;
        epilogue_target(P, split, C, ldc, scale);
        if constexpr (Cfg::F32) tile_epilogue<Cfg>(C, ldc, P.m, P.n, m0, n0, scale, acc);
        else if constexpr (Cfg::M16) lp2_epilogue16<Cfg>(C, ldc, P.m, P.n, m0, n0, scale, acc);
        else lp2_epilogue<Cfg>(C, ldc, P.m, P.n, m0, n0, scale, acc);
    }
}

template <int MODE, int BM, int BN, int STAGES, int WM, int WN, int AROWB, int LDB, int MB>
__device__ __forceinline__ void Lp2Cfg<MODE, BM, BN, STAGES, WM, WN, AROWB, LDB, MB>::run(const TileProblem &P,
                                                                                    int tm, int tn, int split,
                                                                                    uint8_t *lds) {
    lp2_tile<Lp2Cfg<MODE, BM, BN, STAGES, WM, WN, AROWB, LDB, MB>>(P, tm, tn, split, lds);
}
