// Binary64 output tile of C = A*B on gfx950 matrix cores
// (v_mfma_f64_16x16x4_f64).  The paper times the product for double
// matrices as well as float (Results section, Table 2's double column).
//
// Same structure as the FP32 tile: one workgroup of WM x WN waves owns a BM x
// BN tile of C and walks k in k-tiles of BK = 16 doubles through
// two LDS stages (16-byte global loads staged in registers), one barrier per
// k-tile.  A k-tile is 128 bytes per row, as in the FP32 and
// reduced-precision tiles.  A rows are not padded but XOR-swizzled in 16-byte
// chunks (chunk c of row r sits at c ^ ((r >> 1) & 7)): a 16-lane phase of a
// fragment read (16 rows, one chunk each) and of a staging write (2 rows, 8
// chunks each) then both cover 16 distinct 16-byte bank groups.  B rows are
// padded by 16 bytes; their reads and writes cover whole rows.
//
// MFMA operand layout (16x16x4, f64): lane l supplies A[l%16][kslot(l/16)]
// and B[kslot(l/16)][l%16]; the 16x16 result has, in lane l and register r,
// row l/16 + 4*r and column l%16 (measured on gfx950 with an in-bounds probe
// of the instruction; this differs from the 4*(l/16) + r row order of the
// 16x16 float32 forms).
//
// k order: MFMA step t (0..3) of a k-tile chunk of 16 consumes k = 4g + t in
// lane group g = l/16, so that each lane reads its four A values of the
// chunk with two 16-byte LDS reads.  Columns: lane l%16 = jj of a wave owning
// TN = 16*CB columns feeds accumulator block cb = 2h + e with output column
// 32h + 2jj + e (CB = 1: column jj).  Each lane thus reads, and the epilogue
// stores, pairs of consecutive doubles, and the 16 lanes of one row read 256
// contiguous bytes per instruction, which spreads them over all LDS banks.
//
// The C pointer of the TileProblem holds double elements for this tile.
#pragma once

#include "tile_common.hpp"

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int CB> struct DVec;
template <> struct DVec<1> { typedef double T; };
template <> struct DVec<2> { typedef f64x2 T; };
template <> struct DVec<4> { typedef f64x4 T; };

template <int BM_, int BN_, int WM_ = 2, int WN_ = 2>
struct F64Cfg {
    static constexpr int BM = BM_, BN = BN_, BK = 16;
    static constexpr int WM = WM_, WN = WN_;          // waves along m and n
    static constexpr int THREADS = 64 * WM * WN;
    static constexpr int TM = BM / WM, TN = BN / WN;
    static constexpr int RB = TM / 16, CB = TN / 16;
    static constexpr int SA = BK;       // LDS row stride of A (doubles), swizzled
    __device__ static __forceinline__ int a_swz(int r) { return (r >> 1) & 7; }
    static constexpr int SB = BN + 2;   // LDS row stride of B (doubles)
    static constexpr int A_ELEMS = BM * SA, B_ELEMS = BK * SB;
    static constexpr int STAGE = A_ELEMS + B_ELEMS;
    static constexpr int LDS_BYTES = 2 * STAGE * 8;
    static constexpr int AV = BM * BK / 2 / THREADS;  // 16-byte loads per thread (A)
    static constexpr int BV = BK * BN / 2 / THREADS;  // 16-byte loads per thread (B)
    static_assert(RB >= 1 && (CB == 1 || CB == 2 || CB == 4), "wave tile");
    static_assert(AV >= 1 && BV >= 1, "tile too small for the workgroup");
    static_assert(LDS_BYTES <= 160 * 1024, "LDS");
    static constexpr int MFMA_K = 4;
    __device__ static void run(const TileProblem &P, int tm, int tn, int split, uint8_t *lds);
};

// Two consecutive doubles of row r from column c, zero outside [0,R) x [0,Cn).
__device__ __forceinline__ f64x2 f64_load2(const double *__restrict__ P, int64_t ld, int r, int c, int R, int Cn) {
    f64x2 v = {0.0, 0.0};
    if (r < R) {
        const double *p = P + (int64_t)r * ld + c;
        if (c + 1 < Cn) {
            v = __builtin_bit_cast(f64x2, ld16(p));
        } else if (c < Cn) {
            v[0] = p[0];
        }
    }
    return v;
}

template <class Cfg>
__device__ __forceinline__ void f64_load_tiles(const TileProblem &P, int m0, int n0, int k0, f64x2 (&ra)[Cfg::AV],
                                               f64x2 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    const double *A = static_cast<const double *>(P.A);
    const double *B = static_cast<const double *>(P.B);
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 2);
        const int kv = (idx % (Cfg::BK / 2)) * 2;
        ra[q] = f64_load2(A, P.lda, m0 + r, k0 + kv, P.m, P.k);
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 2);
        const int cv = (idx % (Cfg::BN / 2)) * 2;
        rb[q] = f64_load2(B, P.ldb, k0 + kr, n0 + cv, P.k, P.n);
    }
}

template <class Cfg>
__device__ __forceinline__ void f64_store_tiles(double *stage, const f64x2 (&ra)[Cfg::AV],
                                                const f64x2 (&rb)[Cfg::BV]) {
    const int tid = threadIdx.x;
    double *As = stage;
    double *Bs = stage + Cfg::A_ELEMS;
#pragma unroll
    for (int q = 0; q < Cfg::AV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int r = idx / (Cfg::BK / 2);
        const int c = idx % (Cfg::BK / 2);
        *reinterpret_cast<f64x2 *>(&As[r * Cfg::SA + 2 * (c ^ Cfg::a_swz(r))]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < Cfg::BV; ++q) {
        const int idx = tid + q * Cfg::THREADS;
        const int kr = idx / (Cfg::BN / 2);
        const int cv = (idx % (Cfg::BN / 2)) * 2;
        *reinterpret_cast<f64x2 *>(&Bs[kr * Cfg::SB + cv]) = rb[q];
    }
}

template <class Cfg>
__device__ __forceinline__ void f64_compute_stage(const double *stage, f64x4 (&acc)[Cfg::RB][Cfg::CB]) {
    typedef typename DVec<Cfg::CB>::T BVec;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l16 = lane & 15, g = lane >> 4;
    static_assert(Cfg::BK == 16, "one 16-k chunk per k-tile (the swizzle covers 8 chunks)");
    const int ar = wm * Cfg::TM + l16;   // row of block rb is ar + 16 rb: same (r >> 1) & 7
    const double *As = stage + ar * Cfg::SA;
    const int c0 = (2 * g) ^ Cfg::a_swz(ar), c1 = (2 * g + 1) ^ Cfg::a_swz(ar);
    const double *Bs = stage + Cfg::A_ELEMS + (4 * g) * Cfg::SB + wn * Cfg::TN + (Cfg::CB == 1 ? l16 : 2 * l16);
#pragma unroll
    for (int kc = 0; kc < Cfg::BK / 16; ++kc) {
        f64x2 af[Cfg::RB][2];
#pragma unroll
        for (int rb = 0; rb < Cfg::RB; ++rb) {
            const double *p = As + rb * 16 * Cfg::SA;
            af[rb][0] = *reinterpret_cast<const f64x2 *>(p + 2 * c0);
            af[rb][1] = *reinterpret_cast<const f64x2 *>(p + 2 * c1);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // B values of step t, read just before use (fewer live registers)
            BVec bft;
            {
                const double *p = Bs + (kc * 16 + t) * Cfg::SB;
                if constexpr (Cfg::CB == 4) {
                    const f64x2 lo = *reinterpret_cast<const f64x2 *>(p);
                    const f64x2 hi = *reinterpret_cast<const f64x2 *>(p + 32);
                    bft = f64x4{lo[0], lo[1], hi[0], hi[1]};
                } else {
                    bft = *reinterpret_cast<const BVec *>(p);
                }
            }
            BVec bf[4];
            bf[t] = bft;
#pragma unroll
            for (int rb = 0; rb < Cfg::RB; ++rb) {
                const double av = af[rb][t >> 1][t & 1];
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb) {
                    double bv;
                    if constexpr (Cfg::CB == 1) bv = bf[t];
                    else bv = bf[t][cb];
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[rb][cb], 0, 0, 0);
                }
            }
        }
    }
}

template <class Cfg>
__device__ __forceinline__ void f64_epilogue(double *__restrict__ C, int64_t ldc, int M, int N, int m0, int n0,
                                             const f64x4 (&acc)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l16 = lane & 15, g = lane >> 4;
    constexpr int PAIRS = Cfg::CB == 1 ? 1 : Cfg::CB / 2;   // column pairs per lane
    constexpr int PW = Cfg::CB == 1 ? 1 : 2;                // doubles per pair
    const int col0 = n0 + wn * Cfg::TN + (Cfg::CB == 1 ? l16 : 2 * l16);
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + wm * Cfg::TM + rb * 16 + g + 4 * r;
            if (row >= M) continue;
#pragma unroll
            for (int h = 0; h < PAIRS; ++h) {
                const int col = col0 + 32 * h;
                double v[PW];
#pragma unroll
                for (int e = 0; e < PW; ++e) v[e] = acc[rb][PW * h + e][r];
                double *p = C + (int64_t)row * ldc + col;
                if (col + PW <= N) {
                    __builtin_memcpy(p, v, sizeof(v));
                } else {
#pragma unroll
                    for (int e = 0; e < PW; ++e)
                        if (col + e < N) p[e] = v[e];
                }
            }
        }
    }
}

template <class Cfg>
__device__ __forceinline__ void f64_tile(const TileProblem &P, int tm, int tn, double *lds) {
    const int m0 = tm * Cfg::BM, n0 = tn * Cfg::BN;
    const int nkt = (P.k + Cfg::BK - 1) / Cfg::BK;

    f64x4 acc[Cfg::RB][Cfg::CB];
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < Cfg::CB; ++cb) acc[rb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};

    f64x2 ra[Cfg::AV], rbv[Cfg::BV];
    if (nkt > 0) {
        f64_load_tiles<Cfg>(P, m0, n0, 0, ra, rbv);
        f64_store_tiles<Cfg>(lds, ra, rbv);
    }
    __syncthreads();
    for (int kt = 0; kt < nkt; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nkt;
        if (more) f64_load_tiles<Cfg>(P, m0, n0, (kt + 1) * Cfg::BK, ra, rbv);
        f64_compute_stage<Cfg>(lds + cur * Cfg::STAGE, acc);
        if (more) f64_store_tiles<Cfg>(lds + (cur ^ 1) * Cfg::STAGE, ra, rbv);
        __syncthreads();
    }
    f64_epilogue<Cfg>(reinterpret_cast<double *>(P.C), P.ldc, P.m, P.n, m0, n0, acc);
}

template <int BM, int BN, int WM, int WN>
__device__ __forceinline__ void F64Cfg<BM, BN, WM, WN>::run(const TileProblem &P, int tm, int tn, int,
                                                            uint8_t *lds) {
    f64_tile<F64Cfg<BM, BN, WM, WN>>(P, tm, tn, reinterpret_cast<double *>(lds));
}
