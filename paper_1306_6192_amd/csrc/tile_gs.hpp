// Grouped persistent launch with a streamed operand pipeline.
//
// Many independent products (any shapes, any strides and alignments) in one
// launch.  The host lays every output tile of every problem out on a static
// schedule (an ordered tile list per workgroup, see grouped.cpp); each
// workgroup walks its list as one stream of k-tiles and keeps the next
// DEPTH-1 k-tiles of that stream in flight in a ring of register sets while
// it multiplies the current one, across tile boundaries: the first k-tiles of
// the next output tile are already loading while the current tile finishes,
// so no tile pays the full HBM latency of its first k-tile.
//
// Per k-tile of the stream (one step):
//   1. issue the 16-byte global loads of the k-tile DEPTH-1 steps ahead into
//      its register set (always the same number of loads per k-tile, so that
//      one vmcnt wait retires exactly the oldest set);
//   2. multiply the current k-tile from LDS (the register-staged tiles' MFMA
//      code, so the arithmetic and the bits are those of the plain launch of
//      the same configuration);
//   3. wait for the next k-tile's set, fix up its edge chunks (zero past k,
//      realign the chunks read at clamped addresses) and write it to the
//      other LDS stage (the register-staged tiles' LDS layout);
//   4. after the last k-tile of an output tile, store its accumulators;
//   5. one workgroup barrier.
//
// Loads never leave the operands: rows of A past m and columns of B past n
// read clamped (valid) addresses whose results are never stored; k past the
// end is zeroed after the load.  A 16-byte chunk that would run past the end
// of a row is read from the row's other chunks' memory when another row
// follows it in the matrix (rows are lda >= k apart, so the bytes exist),
// and, in the matrix's last row only, read at the last whole chunk of the row
// and shifted into place.  Problems whose k or n is below one chunk (16 bytes
// of elements) take element-wise loads and a full wait instead.
#pragma once

#include <type_traits>

#include "tile_f32.hpp"
#include "tile_lp.hpp"

// s_waitcnt vmcnt(N), the other counters left alone (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt_gs() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Register-staged tile configurations as the stream sees them: NA A-vectors
// and NB B-vectors of 16 bytes per thread per k-tile, the tile-relative
// position of each, and the LDS store / multiply / epilogue of the
// configuration.
template <class Cfg> struct GsOps;

template <int BM, int BN, int WM, int WN, int BK>
struct GsOps<F32Cfg<BM, BN, WM, WN, BK>> {
    typedef F32Cfg<BM, BN, WM, WN, BK> Cfg;
    static constexpr int ESZ = 4;
    static constexpr int NA = Cfg::AV, NB = Cfg::BV;
    typedef f32x16 Acc[Cfg::RB][Cfg::CB];
    // A vector q: tile row r, k offset c; B vector q: k offset kr, tile column c
    __device__ static __forceinline__ void a_pos(int q, int &r, int &c) {
        const int idx = threadIdx.x + q * Cfg::THREADS;
        r = idx / (BK / 4);
        c = (idx % (BK / 4)) * 4;
    }
    __device__ static __forceinline__ void b_pos(int q, int &kr, int &c) {
        const int idx = threadIdx.x + q * Cfg::THREADS;
        kr = idx / (BN / 4);
        c = (idx % (BN / 4)) * 4;
    }
    __device__ static __forceinline__ void store(uint8_t *stage, const u32x4 *v) {
        f32x4 ra[NA], rb[NB];
#pragma unroll
        for (int q = 0; q < NA; ++q) ra[q] = __builtin_bit_cast(f32x4, v[q]);
#pragma unroll
        for (int q = 0; q < NB; ++q) rb[q] = __builtin_bit_cast(f32x4, v[NA + q]);
        f32_store_tiles<Cfg>(reinterpret_cast<float *>(stage), ra, rb);
    }
    __device__ static __forceinline__ void compute(const uint8_t *stage, Acc &acc) {
        f32_compute_stage<Cfg>(reinterpret_cast<const float *>(stage), acc);
    }
};

template <int MODE, int BM, int BN, int BK>
struct GsOps<LpCfg<MODE, BM, BN, BK>> {
    typedef LpCfg<MODE, BM, BN, BK> Cfg;
    static constexpr int ESZ = Cfg::T::IN_ESZ;
    static constexpr int NA = Cfg::AV, NB = Cfg::TKB;
    typedef f32x16 Acc[Cfg::RB][Cfg::CB];
    __device__ static __forceinline__ void a_pos(int q, int &r, int &c) {
        const int idx = threadIdx.x + q * GEMM_THREADS;
        r = idx / Cfg::VPR;
        c = (idx % Cfg::VPR) * (16 / ESZ);
    }
    __device__ static __forceinline__ void b_pos(int q, int &kr, int &c) {
        const int kb = threadIdx.x % Cfg::KBLK, nb = threadIdx.x / Cfg::KBLK;
        kr = kb * Cfg::TKB + q;
        c = nb * Cfg::VN;
    }
    __device__ static __forceinline__ void store(uint8_t *stage, const u32x4 *v) {
        LpStage<Cfg> R;
#pragma unroll
        for (int q = 0; q < NA; ++q) R.a[q] = v[q];
#pragma unroll
        for (int q = 0; q < NB; ++q) R.b[q] = v[NA + q];
        lp_store_tiles<Cfg>(stage, R);
    }
    __device__ static __forceinline__ void compute(const uint8_t *stage, Acc &acc) {
        lp_compute_stage<Cfg>(stage, acc);
    }
};

// The 16 bytes of v shifted down by `sb` bytes (0..15), zeros shifted in.
__device__ __forceinline__ u32x4 gs_shift_down(const u32x4 &v, int sb) {
    const int sw = sb >> 2, sr = sb & 3;
    const uint32_t w0 = v[0], w1 = v[1], w2 = v[2], w3 = v[3];
    auto pick = [&](int i) -> uint32_t {
        return i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : i == 3 ? w3 : 0u;
    };
    u32x4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbyte(pick(i + sw + 1), pick(i + sw), sr);
    return o;
}

// Keep the first `nb` bytes of v (0..16), zero the rest.
__device__ __forceinline__ u32x4 gs_keep_bytes(const u32x4 &v, int nb) {
    u32x4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int left = nb - 4 * i;
        const uint32_t m = left >= 4 ? 0xFFFFFFFFu : left <= 0 ? 0u : (0xFFFFFFFFu >> (32 - 8 * left));
        o[i] = v[i] & m;
    }
    return o;
}

// Pointers read from the descriptors are kept as global-memory pointers, so
// that accesses through them are global instructions, not flat ones (a flat
// access also counts against the LDS counter, and every LDS wait would then
// wait for the stream's loads too).
typedef __attribute__((address_space(1))) const uint8_t gs_gu8;
typedef __attribute__((address_space(1))) float gs_gf32;
typedef u32x4 gs_u32x4_u __attribute__((aligned(1)));
typedef __attribute__((address_space(1))) const gs_u32x4_u gs_gu32x4;

// 16 bytes from any byte address of global memory (unaligned access is on).
__device__ __forceinline__ u32x4 gs_ld16(gs_gu8 *p) { return *reinterpret_cast<gs_gu32x4 *>(p); }

// 16 bytes of row r from element column c, zero outside [0, R) x [0, Cn),
// element by element (the tiny problems' loads).
template <int ESZ>
__device__ __forceinline__ u32x4 gs_ld16_masked(gs_gu8 *base, int64_t ld, int r, int c, int R, int Cn) {
    constexpr int N = 16 / ESZ;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (r < R) {
        gs_gu8 *p = base + ((int64_t)r * ld + c) * ESZ;
#pragma unroll
        for (int e = 0; e < N; ++e)
            if (c + e < Cn) {
#pragma unroll
                for (int i = 0; i < ESZ; ++i) {
                    const int b = e * ESZ + i;
                    w[b >> 2] |= (uint32_t)p[b] << (8 * (b & 3));
                }
            }
    }
    return (u32x4){w[0], w[1], w[2], w[3]};
}

// The accumulators of one tile to C (the element mapping of tile_epilogue:
// lane l%32 of block cb holds output column CB*(l%32) + cb of the wave's
// columns; register r of the 32x32 block holds row 8(r/4) + 4(l/32) + r%4).
// Each lane's row pointer is computed once; the rows it stores are a fixed
// offset times ldc from it (scalar arithmetic).  An interior tile stores
// without any bound test.
template <class Cfg>
__device__ __forceinline__ void gs_epilogue(gs_gf32 *C, int64_t ldc, int M, int N, int m0, int n0, float scale,
                                            const f32x16 (&acc)[Cfg::RB][Cfg::CB]) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave / Cfg::WN, wn = wave % Cfg::WN;
    const int l32 = lane & 31, g = lane >> 5;
    const int col = n0 + wn * Cfg::TN + Cfg::CB * l32;
    const int row0 = m0 + wm * Cfg::TM + 4 * g;
    gs_gf32 *base = C + (int64_t)row0 * ldc + col;
    if (m0 + Cfg::BM <= M && n0 + Cfg::BN <= N) {
#pragma unroll
        for (int rb = 0; rb < Cfg::RB; ++rb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                gs_gf32 *p = base + (int64_t)(rb * 32 + 8 * (r >> 2) + (r & 3)) * ldc;
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb) p[cb] = acc[rb][cb][r] * scale;
            }
        return;
    }
    const int rows_left = M - row0;
    const bool full_cols = col + Cfg::CB <= N;
#pragma unroll
    for (int rb = 0; rb < Cfg::RB; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int d = rb * 32 + 8 * (r >> 2) + (r & 3);
            if (d >= rows_left) continue;
            gs_gf32 *p = base + (int64_t)d * ldc;
            if (full_cols) {
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb) p[cb] = acc[rb][cb][r] * scale;
            } else {
#pragma unroll
                for (int cb = 0; cb < Cfg::CB; ++cb)
                    if (col + cb < N) p[cb] = acc[rb][cb][r] * scale;
            }
        }
    }
}

// What the stream reads about one output tile: its schedule entry and its
// problem's descriptor, through restrict-qualified pointers with a
// wave-uniform index, so that the compiler keeps them in scalar registers
// (scalar loads; no vector-memory wait).
struct GsTile {
    gs_gu8 *A, *B;
    gs_gf32 *C;
    int64_t lda, ldb, ldc;
    int m, n, k;
    float scale;
    int cfg;        // 0 or 1
    int m0, n0;
    int nkt;        // k-tiles of the tile's configuration (at least 1)
    int tiny;       // k or n below one 16-byte chunk: element-wise loads
};

template <int ESZ>
__device__ __forceinline__ GsTile gs_tile(const GroupDesc *__restrict__ descs, const GroupTile *__restrict__ tiles,
                                          int i) {
    const GroupTile e = tiles[__builtin_amdgcn_readfirstlane(i)];
    const GroupDesc &d = descs[__builtin_amdgcn_readfirstlane(e.p)];
    GsTile T;
    T.A = (gs_gu8 *)d.P.A;
    T.B = (gs_gu8 *)d.P.B;
    T.C = (gs_gf32 *)d.P.C;
    T.lda = d.P.lda;
    T.ldb = d.P.ldb;
    T.ldc = d.P.ldc;
    T.m = d.P.m;
    T.n = d.P.n;
    T.k = d.P.k;
    T.scale = d.P.scale;
    T.cfg = d.cfg;
    T.m0 = e.m0;
    T.n0 = e.n0;
    T.nkt = e.nkt;
    T.tiny = T.k < 16 / ESZ || T.n < 16 / ESZ;
    return T;
}

// What the multiply cursor keeps of its tile from one k-tile to the next
// (the bounds the staging needs); the operands and C are read from the
// schedule where they are needed (tiny tiles, the epilogue).
struct GsCur {
    int m, n, k, m0, n0, cfg, nkt, tiny;
};

template <int ESZ>
__device__ __forceinline__ GsCur gs_cur(const GroupDesc *__restrict__ descs, const GroupTile *__restrict__ tiles,
                                        int i) {
    const GsTile T = gs_tile<ESZ>(descs, tiles, i);
    return GsCur{T.m, T.n, T.k, T.m0, T.n0, T.cfg, T.nkt, T.tiny};
}

// Source addresses of the NV loads of k-tile kt of tile T for configuration
// Cfg (see the file comment for the addresses).
template <class Cfg, int NV>
__device__ __forceinline__ void gs_addr_cfg(const GsTile &T, int kt, gs_gu8 *(&src)[NV]) {
    typedef GsOps<Cfg> O;
    static_assert(O::NA + O::NB == NV, "one load count per grouped kernel");
    constexpr int ESZ = O::ESZ, CE = 16 / ESZ;
    const int k0 = kt * Cfg::BK;
    const bool ktail = k0 + Cfg::BK > T.k;
#pragma unroll
    for (int q = 0; q < O::NA; ++q) {
        int r, c;
        O::a_pos(q, r, c);
        const int row = min(T.m0 + r, T.m - 1);
        int col = k0 + c;
        // a chunk wholly past k, or the last row's chunk that runs past k:
        // read the row's last whole chunk
        if (ktail && col + CE > T.k && (row == T.m - 1 || col >= T.k)) col = T.k - CE;
        src[q] = T.A + ((int64_t)row * T.lda + col) * ESZ;
    }
    const bool nedge = T.n0 + Cfg::BN > T.n;
#pragma unroll
    for (int q = 0; q < O::NB; ++q) {
        int kr, c;
        O::b_pos(q, kr, c);
        const int krow = min(k0 + kr, T.k - 1);
        int col = T.n0 + c;
        // a chunk wholly past n, or the last row's chunk that runs past n:
        // read the row's last whole chunk
        if (nedge && col + CE > T.n && (krow == T.k - 1 || col >= T.n)) col = T.n - CE;
        src[O::NA + q] = T.B + ((int64_t)krow * T.ldb + col) * ESZ;
    }
}

// Element-wise, masked loads of k-tile kt of a tiny tile (k or n below one
// chunk), completed before return.
template <class Cfg, int NV>
__device__ __forceinline__ void gs_load_tiny(const GsTile &T, int kt, u32x4 (&v)[NV]) {
    typedef GsOps<Cfg> O;
    constexpr int ESZ = O::ESZ;
    const int k0 = kt * Cfg::BK;
#pragma unroll
    for (int q = 0; q < O::NA; ++q) {
        int r, c;
        O::a_pos(q, r, c);
        v[q] = gs_ld16_masked<ESZ>(T.A, T.lda, T.m0 + r, k0 + c, T.m, T.k);
    }
#pragma unroll
    for (int q = 0; q < O::NB; ++q) {
        int kr, c;
        O::b_pos(q, kr, c);
        v[O::NA + q] = gs_ld16_masked<ESZ>(T.B, T.ldb, k0 + kr, T.n0 + c, T.k, T.n);
    }
    wait_vmcnt_gs<0>();
}

// Fix up the edge chunks of k-tile kt of tile T after they have landed:
// zero A past k, zero B rows past k, and shift the chunks read at a clamped
// column into place.
template <class Cfg, class TT, int NV>
__device__ __forceinline__ void gs_fixup_cfg(const TT &T, int kt, u32x4 (&v)[NV]) {
    typedef GsOps<Cfg> O;
    constexpr int ESZ = O::ESZ, CE = 16 / ESZ;
    const int k0 = kt * Cfg::BK;
    if (k0 + Cfg::BK > T.k) {
#pragma unroll
        for (int q = 0; q < O::NA; ++q) {
            int r, c;
            O::a_pos(q, r, c);
            const int row = min(T.m0 + r, T.m - 1);
            const int col = k0 + c;
            u32x4 x = v[q];
            if (row == T.m - 1 && col + CE > T.k && col < T.k) x = gs_shift_down(x, (col - (T.k - CE)) * ESZ);
            v[q] = gs_keep_bytes(x, max(0, min(CE, T.k - col)) * ESZ);
        }
#pragma unroll
        for (int q = 0; q < O::NB; ++q) {
            int kr, c;
            O::b_pos(q, kr, c);
            if (k0 + kr >= T.k) v[O::NA + q] = (u32x4){0u, 0u, 0u, 0u};
        }
    }
    if (T.n0 + Cfg::BN > T.n) {
#pragma unroll
        for (int q = 0; q < O::NB; ++q) {
            int kr, c;
            O::b_pos(q, kr, c);
            const int col = T.n0 + c;
            if (k0 + kr == T.k - 1 && col < T.n && col + CE > T.n)
                v[O::NA + q] = gs_shift_down(v[O::NA + q], (col - (T.n - CE)) * ESZ);
        }
    }
}

template <class C0, class C1>
struct GsRing {
    static constexpr int NV = GsOps<C0>::NA + GsOps<C0>::NB;
    static_assert(GsOps<C1>::NA + GsOps<C1>::NB == NV, "both tiles load the same number of 16-byte vectors");
    static constexpr int STAGE0 = C0::LDS_BYTES / 2, STAGE1 = C1::LDS_BYTES / 2;
    static constexpr int STAGE = STAGE0 > STAGE1 ? STAGE0 : STAGE1;
    static constexpr int ESZ = GsOps<C0>::ESZ;
    static_assert(GsOps<C0>::ESZ == GsOps<C1>::ESZ, "one element type per grouped kernel");
    static constexpr bool ONE = std::is_same<C0, C1>::value;   // one tile configuration
};

// The stream's state: the lookahead cursor (li, lkt: the next k-tile to
// load; LT: its tile; src: the per-lane addresses of the k-tile it loaded
// last) runs DEPTH-1 k-tiles ahead of the multiply cursor (ci, ckt; CT: its
// tile); `step` counts the k-tiles multiplied.  A cursor reads its tile's
// record from the schedule only when it enters the tile.
template <int NV>
struct GsState {
    int li, lkt, ci, ckt, step;
    GsTile LT;
    GsCur CT;
    gs_gu8 *src[NV];
};

// Advance the addresses of the NV loads by one k-tile (an interior k-tile:
// no bound depends on k there, so each address moves by the k-tile's
// stride: BK elements along an A row, BK rows down B).
template <class Cfg, int NV>
__device__ __forceinline__ void gs_advance_cfg(const GsTile &T, gs_gu8 *(&src)[NV]) {
    typedef GsOps<Cfg> O;
#pragma unroll
    for (int q = 0; q < O::NA; ++q) src[q] += Cfg::BK * O::ESZ;
    const int64_t bstep = (int64_t)Cfg::BK * T.ldb * O::ESZ;
#pragma unroll
    for (int q = 0; q < O::NB; ++q) src[O::NA + q] += bstep;
}

// Issue the lookahead k-tile into ring set `v` and advance the lookahead.
// Straight-line: every call issues exactly NV 16-byte loads, so that the
// ring registers are only ever written by these loads (no merge of register
// values across branches, which would make the compiler copy -- and so wait
// for -- a set still in flight) and one vmcnt count retires the oldest set.
// Past the end of the list, and for tiny tiles (loaded element-wise when
// they reach the LDS), the loads read a valid dummy address (the schedule's
// first entry).  The addresses are computed in full at a tile's first and
// last k-tile and advanced by one k-tile in between.
template <class C0, class C1, int NV>
__device__ __forceinline__ void gs_lookahead(const GroupDesc *__restrict__ descs,
                                             const GroupTile *__restrict__ tiles, int last, GsState<NV> &s,
                                             u32x4 (&v)[NV]) {
    typedef GsRing<C0, C1> R;
    const bool real = s.li < last;
    // s.src holds the dummy address for a tiny tile and past the end of the
    // list (set when the cursor gets there), so the loads need no select
    if (real && !s.LT.tiny) {
        const bool first_cfg = R::ONE || s.LT.cfg == 0;
        if (s.lkt == 0 || s.lkt + 1 == s.LT.nkt) {
            if (first_cfg) gs_addr_cfg<C0>(s.LT, s.lkt, s.src);
            else gs_addr_cfg<C1>(s.LT, s.lkt, s.src);
        } else {
            if (first_cfg) gs_advance_cfg<C0>(s.LT, s.src);
            else gs_advance_cfg<C1>(s.LT, s.src);
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = gs_ld16(s.src[q]);
    if (real && ++s.lkt == s.LT.nkt) {
        s.lkt = 0;
        if (++s.li < last) s.LT = gs_tile<R::ESZ>(descs, tiles, s.li);
        if (s.li >= last || s.LT.tiny) {
#pragma unroll
            for (int q = 0; q < NV; ++q) s.src[q] = (gs_gu8 *)tiles;
        }
    }
}

// The k-tile kt of tile i of the schedule (bounds in `T`; data in ring set
// `v`, already waited for; the set is free afterwards) into the LDS stage
// `dst`.  Tiny tiles read their operands element-wise here.
template <class C0, class C1, int NV>
__device__ __forceinline__ void gs_stage(const GroupDesc *__restrict__ descs, const GroupTile *__restrict__ tiles,
                                         int i, const GsCur &T, int kt, u32x4 (&v)[NV], uint8_t *dst) {
    if (T.tiny) {
        const GsTile F = gs_tile<GsRing<C0, C1>::ESZ>(descs, tiles, i);
        if (GsRing<C0, C1>::ONE || T.cfg == 0) gs_load_tiny<C0>(F, kt, v);
        else gs_load_tiny<C1>(F, kt, v);
    } else {
        if (GsRing<C0, C1>::ONE || T.cfg == 0) gs_fixup_cfg<C0>(T, kt, v);
        else gs_fixup_cfg<C1>(T, kt, v);
    }
    if (GsRing<C0, C1>::ONE || T.cfg == 0) GsOps<C0>::store(dst, v);
    else GsOps<C1>::store(dst, v);
}

// One step of the stream: U is the step's position in the DEPTH-unrolled
// loop (its register sets are ring[(U + DEPTH - 1) % DEPTH] for the issue and
// ring[(U + 1) % DEPTH] for the next k-tile).  Returns false when the
// workgroup's list is done.
template <class C0, class C1, int DEPTH, int U>
__device__ __forceinline__ bool gs_step(const GroupDesc *__restrict__ descs, const GroupTile *__restrict__ tiles,
                                        int last, uint8_t *lds, u32x4 (&ring)[DEPTH][GsRing<C0, C1>::NV],
                                        GsState<GsRing<C0, C1>::NV> &s, typename GsOps<C0>::Acc &acc0,
                                        typename GsOps<C1>::Acc &acc1) {
    typedef GsRing<C0, C1> R;
    uint8_t *cur = lds + (s.step & 1) * R::STAGE;
    uint8_t *nxt = lds + ((s.step + 1) & 1) * R::STAGE;
    // 1. the k-tile DEPTH-1 steps ahead
    gs_lookahead<C0, C1>(descs, tiles, last, s, ring[(U + DEPTH - 1) % DEPTH]);
    const bool tile_end = s.ckt + 1 == s.CT.nkt;
    const int ni = tile_end ? s.ci + 1 : s.ci;
    const int nk = tile_end ? 0 : s.ckt + 1;
    // the next tile's bounds (read while the current k-tile is multiplied)
    GsCur NT = s.CT;
    if (tile_end && ni < last) NT = gs_cur<R::ESZ>(descs, tiles, ni);
    // 2. the current k-tile
    if (R::ONE || s.CT.cfg == 0) GsOps<C0>::compute(cur, acc0);
    else GsOps<C1>::compute(cur, acc1);
    // 3. the next k-tile into the other LDS stage: its set is the oldest in
    // flight, DEPTH-2 sets (all issued, real or dummy) came after it
    wait_vmcnt_gs<(DEPTH - 2) * R::NV>();
    if (ni < last) gs_stage<C0, C1>(descs, tiles, ni, NT, nk, ring[(U + 1) % DEPTH], nxt);
    // 4. the finished tile's accumulators
    if (tile_end) {
        const GsTile CT = gs_tile<R::ESZ>(descs, tiles, s.ci);
        if (R::ONE || CT.cfg == 0) {
            gs_epilogue<C0>(CT.C, CT.ldc, CT.m, CT.n, CT.m0, CT.n0, CT.scale, acc0);
#pragma unroll
            for (int rb = 0; rb < C0::RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < C0::CB; ++cb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc0[rb][cb][r] = 0.f;
        } else {
            gs_epilogue<C1>(CT.C, CT.ldc, CT.m, CT.n, CT.m0, CT.n0, CT.scale, acc1);
#pragma unroll
            for (int rb = 0; rb < C1::RB; ++rb)
#pragma unroll
                for (int cb = 0; cb < C1::CB; ++cb)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc1[rb][cb][r] = 0.f;
        }
        s.CT = NT;
    }
    // keep this step's set (staged one step ago, reloaded by the next step)
    // live until the reload, so that its registers are not lent to
    // temporaries, which would have to wait for its load
#pragma unroll
    for (int q = 0; q < R::NV; ++q) asm volatile("" ::"v"(ring[U % DEPTH][q]));
    __syncthreads();
    ++s.step;
    s.ci = ni;
    s.ckt = nk;
    return ni < last;
}

// The persistent kernel: workgroup w walks tiles [wg_first[w], wg_first[w+1])
// of the schedule.  C0 and C1 are register-staged tile configurations of one
// mode (the descriptor's cfg picks one per problem).
template <class C0, class C1, int OCC, int DEPTH>
__global__ __launch_bounds__(GEMM_THREADS, OCC) void gemm_grouped_stream_kernel(
    const GroupDesc *__restrict__ descs, const GroupTile *__restrict__ tiles, const int32_t *__restrict__ wg_first) {
    static_assert(C0::THREADS == GEMM_THREADS && C1::THREADS == GEMM_THREADS, "256-lane tiles");
    typedef GsRing<C0, C1> R;
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * R::STAGE];
    const int first = wg_first[blockIdx.x], last = wg_first[blockIdx.x + 1];
    if (first >= last) return;

    // C1's accumulators are C0's first block when C1 has one block per wave
    // (the two tiles never run at once, and each leaves its accumulators at
    // zero for the next tile): sixteen registers fewer
    typename GsOps<C0>::Acc acc0;
    constexpr bool SHARE = !R::ONE && C1::RB == 1 && C1::CB == 1;
    typename GsOps<C1>::Acc acc1_own;
    typename GsOps<C1>::Acc &acc1 =
        SHARE ? *reinterpret_cast<typename GsOps<C1>::Acc *>(&acc0[0][0]) : acc1_own;
#pragma unroll
    for (int rb = 0; rb < C0::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < C0::CB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc0[rb][cb][r] = 0.f;
    if constexpr (!SHARE) {
#pragma unroll
        for (int rb = 0; rb < C1::RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < C1::CB; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc1[rb][cb][r] = 0.f;
    }

    u32x4 ring[DEPTH][R::NV];
    GsState<R::NV> s;
    s.li = s.ci = first;
    s.lkt = s.ckt = s.step = 0;
    s.LT = gs_tile<R::ESZ>(descs, tiles, first);
    s.CT = gs_cur<R::ESZ>(descs, tiles, first);
    // the dummy address until the lookahead computes the first tile's
    // addresses (and for good if that tile is tiny)
#pragma unroll
    for (int q = 0; q < R::NV; ++q) s.src[q] = (gs_gu8 *)tiles;
    // prologue: k-tiles 0 .. DEPTH-2 of the stream in flight, k-tile 0 in LDS
#pragma unroll
    for (int u = 0; u < DEPTH - 1; ++u) gs_lookahead<C0, C1>(descs, tiles, last, s, ring[u]);
    wait_vmcnt_gs<(DEPTH - 2) * R::NV>();
    gs_stage<C0, C1>(descs, tiles, first, s.CT, 0, ring[0], lds);
    __syncthreads();
    // steady state: step j multiplies stream k-tile j (ring set j % DEPTH)
    while (true) {
        if (!gs_step<C0, C1, DEPTH, 0>(descs, tiles, last, lds, ring, s, acc0, acc1)) break;
        if constexpr (DEPTH > 1)
            if (!gs_step<C0, C1, DEPTH, 1 % DEPTH>(descs, tiles, last, lds, ring, s, acc0, acc1)) break;
        if constexpr (DEPTH > 2)
            if (!gs_step<C0, C1, DEPTH, 2 % DEPTH>(descs, tiles, last, lds, ring, s, acc0, acc1)) break;
        if constexpr (DEPTH > 3)
            if (!gs_step<C0, C1, DEPTH, 3 % DEPTH>(descs, tiles, last, lds, ring, s, acc0, acc1)) break;
        if constexpr (DEPTH > 4)
            if (!gs_step<C0, C1, DEPTH, 4 % DEPTH>(descs, tiles, last, lds, ring, s, acc0, acc1)) break;
    }
}
