// Dense contraction steps on the matrix cores for residues modulo small
// moduli (m <= 255), stored as centred int8 values (|r| <= 127).
//
// A step C = A B^T (rows of A and B contiguous along the shared bonds, Sec.
// 2.1 / Eq. 5 in the plan's layout) is an int8 matrix product: every
// product of two residues is at most 127^2 < 2^14 in magnitude, so
// v_mfma_i32_16x16x64_i8 sums 2^16 of them exactly in int32 (< 2^30); wider
// K is reduced to a centred residue every 2^16 entries. The epilogue reduces
// each sum modulo m (ModSmall) and stores the int8 residue, which the next
// step reads as it is: no digit pass and one product per multiply-add.
//
// Work-group tile WM (xA) x WN (xB) with waves of 16 RA x 16 CB outputs:
// 8 waves (two per SIMD) on 256 x 256 tiles when both free sides have 8
// bits, else 256 x 128 or 128 x 128; 4 waves on 256 x 64 or 128 x 64 tiles
// when B's free side has 6 bits (those steps stream A at the memory rate). K goes in stages of one 64-entry
// chunk: 64-byte LDS rows, filled straight from global memory
// (global_load_lds_dwordx4, 16 rows per wave instruction) through four
// buffers; stage k+4 is requested while stage k is multiplied, and at a
// tile's last stage (every fragment in registers) the next tile's first
// four stages. One barrier per stage; after it the wave reads the next
// stage's fragments while the current stage's MFMAs run.
//
// LDS rows: 4 slots of 16 bytes, slot c of row r stored at slot
// c ^ ((r / 2) % 4). A 16-byte read is served eight lanes at a time, and
// eight lanes free of bank conflicts cover 128 distinct bytes modulo 128. A
// fragment read has eight consecutive lanes on eight consecutive rows at one
// logical slot: rows of one parity lie 128 bytes apart, and (r / 2) % 4 sends
// the four rows of each parity to four distinct slots. (Measured on gfx950:
// 212 B/clk per CU with this map, 124 B/clk with c ^ ((r / 4) % 4), whose
// eight lanes meet in pairs.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "mfma.hpp"
#include "mfma_common.hpp"
#include "profile.hpp"
#include "tune.hpp"

namespace tn {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int k8Row = 64;                  // LDS row bytes: one 64-entry chunk
constexpr int k8Bufs = 4;
constexpr int k8Flush = (1 << 16) / 64;    // chunks per exact int32 range
constexpr int k8MaxRowBytesLog = 25;       // 127 rows of a stage within 32-bit load offsets

// Output addressing of the epilogue, by the host: C offset bits of the
// tile-local A indices 16 rb (rb < 8) and v (v < 4) and of the B indices
// 16 cb (cb < 4). A lane holds four outputs, A indices v = 0..3 (A's two
// lowest bits) at one B index. mode 0: those are C's two lowest bits, so
// the four are consecutive bytes; mode 1: C's two lowest bits are A's
// lowest and B's lowest (either order), so a lane and its neighbour (B
// indices differing in the lowest bit) swap halves and each stores 4
// consecutive bytes, the even lane those of v < 2 and the odd lane those of
// v >= 2; sel are the byte selectors of that swap (even, odd lane); mode 2:
// single bytes. In modes 0 and 1, C's bits 2 and 3 then belong to lane bits
// x2 and x3 (B indices' four lowest bits are lane bits 0..3, A indices'
// bits 2 and 3 lane bits 4 and 5, and in mode 1 lane bit 0 stands for A's
// bit 1): exchanging those with two bits of the block index leaves 16
// consecutive bytes of C in each lane (x2 = -1: 4-byte stores).
struct Mfma8Extra {
    uint64_t dA[8], dV[4], dB[4];
    uint32_t sel[2];
    int32_t mode, x2, x3;
    int32_t form;  // 16-byte store variant (store_tile8), 0: none
};

// Centred residue of an exact int32 sum modulo m <= 255, returned as the low
// byte of a word. With FOLD, x = h 2^16 + l becomes y = h (2^16 mod m) + l,
// |y| < 2^15 (m - 1) + 2^16; else the sum covers K <= 512 and
// |y| = |x| <= 512 127^2. Either way |y| < 2^23 is exact in single precision.
// One fma adds y fl(1/m) to 1.5 2^23 and rounds the exact sum once: with
// |y fl(1/m)| < 2^22 the result lies where floats are spaced 1 apart, so its
// low 24 bits, read as a signed 24-bit integer, are 2^22 + q, q the nearest
// integer to y fl(1/m) (ties to even). One 24-bit multiply-add gives
// y - m (2^22 + q) = r - 2^22 m with r = y - q m, whose low byte is r's since
// 256 divides 2^22 m. |r| <= 127 for every m in 2..255 (checked over every
// reachable y), so that byte is r in two's complement.
template <bool FOLD>
__device__ __forceinline__ uint32_t res8(int32_t x, int32_t r16, int32_t negm, float inv) {
    const int32_t y = FOLD ? (x >> 16) * r16 + (x & 0xffff) : x;
    const float u = __builtin_fmaf(float(y), inv, 12582912.0f);
    return uint32_t(__mul24(int32_t(__float_as_uint(u)), negm) + y);
}

// The low bytes of four words, packed (word 0 in byte 0).
__device__ __forceinline__ uint32_t pack4(uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3) {
    const uint32_t lo = __builtin_amdgcn_perm(t1, t0, 0x0c0c0400u), hi = __builtin_amdgcn_perm(t3, t2, 0x0c0c0400u);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// Exchange lane bit k with the index of a pair of words: afterwards the lane
// with bit k = t holds in x (y) the word the lane with bit k = 0 (1) held in
// its word t. P = 4 or 5: lane bit 4 or 5, one permlane swap; P = 0: lane
// bit k < 4 (run-time), a cross-lane read (ds_bpermute) and selects.
template <int P>
__device__ __forceinline__ void lane_swap(uint32_t& x, uint32_t& y, int k, int lane) {
    if constexpr (P == 4 || P == 5) {
        const auto r = P == 4 ? __builtin_amdgcn_permlane16_swap(x, y, false, false)
                              : __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = r[0];
        y = r[1];
    } else {
        const bool hi = (lane >> k) & 1;
        const int send = int(hi ? x : y);
        const int recv = __builtin_amdgcn_ds_bpermute((lane ^ (1 << k)) << 2, send);
        x = hi ? uint32_t(recv) : x;
        y = hi ? y : uint32_t(recv);
    }
}

// The lane's word of block (rb, cb) (see Mfma8Extra): four reduced outputs
// packed; with PAIR, half exchanged with the neighbour lane.
template <int RA, int CB, bool FOLD, bool PAIR>
__device__ __forceinline__ uint32_t out_word(const v4i (&acc)[RA][CB], int rb, int cb, const ModSmall& ms,
                                             uint32_t sel) {
    const int32_t negm = -int32_t(ms.m);
    const int32_t r16 = int32_t(ms.r16);
    const uint32_t x =
        pack4(res8<FOLD>(acc[rb][cb][0], r16, negm, ms.inv), res8<FOLD>(acc[rb][cb][1], r16, negm, ms.inv),
              res8<FOLD>(acc[rb][cb][2], r16, negm, ms.inv), res8<FOLD>(acc[rb][cb][3], r16, negm, ms.inv));
    if constexpr (!PAIR) return x;
    // the neighbour lane's word (quad permutation 1, 0, 3, 2)
    const uint32_t y = uint32_t(__builtin_amdgcn_mov_dpp(int(x), 0xb1, 0xf, 0xf, false));
    return __builtin_amdgcn_perm(x, y, sel);
}

// 16-byte stores: blocks b = rb + RA cb in groups of four (block bits 0 and
// 1) exchange those bits with lane bits x2 and x3 (forms P2, P3 of
// lane_swap); afterwards word t of a group is C's bytes 4t..4t+3 of the
// lane's 16.
template <int RA, int CB, bool FOLD, bool PAIR, int P2, int P3>
__device__ __forceinline__ void store16(const v4i (&acc)[RA][CB], int8_t* C, uint64_t baseC, const Mfma8Extra& ex,
                                        const ModSmall& ms, int lane) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    // (a select: indexing the argument array per lane would load it from
    // memory, and that load's wait would also wait for every load and store
    // in flight)
    const uint32_t sel = (lane & 1) ? ex.sel[1] : ex.sel[0];
#pragma unroll
    for (int g = 0; g < RA * CB; g += 4) {
        uint32_t w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t] = out_word<RA, CB, FOLD, PAIR>(acc, (g + t) % RA, (g + t) / RA, ms, sel);
        lane_swap<P2>(w[0], w[1], ex.x2, lane);
        lane_swap<P2>(w[2], w[3], ex.x2, lane);
        lane_swap<P3>(w[0], w[2], ex.x3, lane);
        lane_swap<P3>(w[1], w[3], ex.x3, lane);
        uint64_t row = baseC | ex.dA[g % RA];
        __asm__ volatile("" : "+v"(row));
        *reinterpret_cast<u4*>(C + (row | ex.dB[g / RA])) = u4{w[0], w[1], w[2], w[3]};
    }
}

// Store a wave's outputs of one tile: lane (fr, q) holds acc[rb][cb][v] for
// A index 16 rb + 4 q + v and B index 16 cb + fr (plus the wave's offsets);
// baseC is the C offset of the lane's first stored byte (tile, wave and lane
// parts, see Mfma8Extra for the modes; form selects the 16-byte variant).
// (Row offsets pass through an empty asm statement so that the compiler does
// not precompute all RA x CB table combinations in scalar registers, which
// would spill.)
template <int RA, int CB, bool FOLD>
__device__ __forceinline__ void store_tile8(const v4i (&acc)[RA][CB], int8_t* C, uint64_t baseC, const Mfma8Extra& ex,
                                            const ModSmall& ms, int lane) {
    switch (ex.form) {
        case 1: return store16<RA, CB, FOLD, false, 4, 5>(acc, C, baseC, ex, ms, lane);
        case 2: return store16<RA, CB, FOLD, false, 4, 0>(acc, C, baseC, ex, ms, lane);
        case 3: return store16<RA, CB, FOLD, false, 0, 4>(acc, C, baseC, ex, ms, lane);
        case 4: return store16<RA, CB, FOLD, false, 0, 0>(acc, C, baseC, ex, ms, lane);
        case 5: return store16<RA, CB, FOLD, true, 0, 4>(acc, C, baseC, ex, ms, lane);
        case 6: return store16<RA, CB, FOLD, true, 0, 0>(acc, C, baseC, ex, ms, lane);
        default: break;
    }
    // (a select: indexing the argument array per lane would load it from
    // memory, and that load's wait would also wait for every load and store
    // in flight)
    const uint32_t sel = (lane & 1) ? ex.sel[1] : ex.sel[0];
    if (ex.mode != 2) {
#pragma unroll
        for (int rb = 0; rb < RA; ++rb) {
            uint64_t row = baseC | ex.dA[rb];
            __asm__ volatile("" : "+v"(row));
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                *reinterpret_cast<uint32_t*>(C + (row | ex.dB[cb])) = out_word<RA, CB, FOLD, true>(acc, rb, cb, ms, sel);
        }
    } else {
        const int32_t negm = -int32_t(ms.m);
        const int32_t r16 = int32_t(ms.r16);
#pragma unroll
        for (int rb = 0; rb < RA; ++rb) {
            uint64_t row = baseC | ex.dA[rb];
            __asm__ volatile("" : "+v"(row));
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    C[row | ex.dV[v] | ex.dB[cb]] = int8_t(res8<FOLD>(acc[rb][cb][v], r16, negm, ms.inv));
        }
    }
}

// Lane part of the C offset of the lane's first stored byte (see Mfma8Extra):
// A index wr + 4 q, B index wc + fr; in mode 1 the lane stores the outputs of
// B index wc + (fr & ~1) and A indices wr + 4 q + 2 (fr & 1) + {0, 1}; with
// 16-byte stores lane bits x2 and x3 stand for block bits 0 and 1 instead
// (rb's bit 0, and rb's bit 1 or, with RA = 2, cb's bit 0).
template <int RA>
__device__ __forceinline__ uint64_t lane_offset8(const StepArgs& a, const Mfma8Extra& ex, int wr, int wc, int lane) {
    uint32_t ai = uint32_t(wr), bi = uint32_t(wc);
    for (int k = 0; k < 6; ++k) {
        if (!((lane >> k) & 1)) continue;
        if (ex.mode != 2 && k == ex.x2)
            ai += 16;
        else if (ex.mode != 2 && k == ex.x3)
            (RA >= 4 ? ai : bi) += RA >= 4 ? 32 : 16;
        else if (k >= 4)
            ai += 4u << (k - 4);
        else if (k == 0 && ex.mode == 1)
            ai += 2;
        else
            bi += 1u << k;
    }
    return pdep64(ai, a.maskA) | pdep64(bi, a.maskB);
}

constexpr int lg2(int x) { return x <= 1 ? 0 : 1 + lg2(x / 2); }

// Tile shape: WM x WN outputs, NW waves, each on 16 RA x 16 CB outputs.
template <int WM_, int WN_, int NW_, int RA_, int CB_>
struct Cfg {
    static constexpr int WM = WM_, WN = WN_, NW = NW_, RA = RA_, CB = CB_;
    static constexpr int THREADS = 64 * NW;
    static constexpr int ROWS = WM + WN;
    static constexpr int BUF = ROWS * k8Row;      // one stage
    static constexpr int GROUP = 16 * NW;         // stage rows per load instruction of all waves
    static constexpr int LOADS = ROWS / GROUP;    // load instructions per wave and stage
    static constexpr int WAVES_A = WM / (16 * RA);
    static constexpr int LGM = lg2(WM), LGN = lg2(WN);
    static_assert(WM % GROUP == 0 && WN % GROUP == 0, "a load instruction covers A rows or B rows only");
    static_assert(WAVES_A * (WN / (16 * CB)) == NW, "waves cover the tile");
};
using Cfg256x256 = Cfg<256, 256, 8, 8, 4>;
using Cfg256x128 = Cfg<256, 128, 8, 8, 2>;
using Cfg128x128 = Cfg<128, 128, 8, 4, 2>;
using Cfg256x64 = Cfg<256, 64, 4, 4, 4>;
using Cfg128x64 = Cfg<128, 64, 4, 2, 4>;

// One step on int8 residues: tiles of WM x WN outputs dealt round-robin to
// the work-groups, K split over blockIdx.y into `splits` ranges (partial
// residues to `part` when splits > 1), residue planes over blockIdx.z.
// NK: 1 or 2 stages per tile and block row, or 4 for any power of two >= 4.
// FOLD: the sums exceed 8 stages, so the epilogue folds them at 2^16 first.
template <class G, int NK, bool FOLD>
__global__ __launch_bounds__(G::THREADS, 1) void k_mfma8(StepArgs a, Mfma8Extra ex, int splits, int8_t* part,
                                                         int64_t part_stride) {
    constexpr int RA = G::RA, CB = G::CB;
    // one LDS buffer per stage in flight: tiles of one or two stages leave
    // room for more work-groups per CU
    constexpr int NBUF = NK < k8Bufs ? NK : k8Bufs;
    __shared__ __align__(1024) uint8_t lds[NBUF * G::BUF + G::THREADS * 8];
    uint64_t* const lconst = reinterpret_cast<uint64_t*>(lds + NBUF * G::BUF);

    const int g = blockIdx.z;
    const int8_t* A = static_cast<const int8_t*>(a.A) + g * a.strideA;
    const int8_t* B = static_cast<const int8_t*>(a.B) + g * a.strideB;
    int8_t* C = static_cast<int8_t*>(a.C) + g * a.strideC;
    const ModSmall ms{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (w % G::WAVES_A) * 16 * RA, wc = (w / G::WAVES_A) * 16 * CB;
    const uint64_t rowBytes = uint64_t(1) << a.s;
    const int nk = NK >= 4 ? (1 << (a.s - 6)) / splits : NK;  // stages per tile and block row
    const int kc0 = int(blockIdx.y) * nk;
    const int lgA = a.fA - G::LGM, lgB = a.fB - G::LGN;
    const uint32_t T = 1u << (lgA + lgB);
    if (blockIdx.x >= T) return;

    const int fr = lane & 15, q = lane >> 4;
    // lane part of the output offset, kept in LDS: the epilogue reads it
    // once per tile, and in registers through the K loop it would only add
    // pressure
    lconst[tid] = lane_offset8<RA>(a, ex, wr, wc, lane);
    // loads: lane l of wave w, instruction i fills physical slot l % 4 of
    // stage row r = GROUP i + 16 w + l / 4, i.e. logical slot
    // (l % 4) ^ ((r / 2) % 4) = (l % 4) ^ ((l / 8) % 4): bytes 16 of that
    // slot of the row's chunk
    const uint32_t voff =
        uint32_t(16 * w + (lane >> 2)) * uint32_t(rowBytes) + 16u * uint32_t((lane & 3) ^ ((lane >> 3) & 3));
    // fragment reads: row wr + fr (A) or WM + wc + fr (B) of a stage, at
    // logical slot q
    const int sw = 16 * (q ^ ((fr >> 1) & 3));
    const uint32_t rdA = uint32_t((wr + fr) * k8Row + sw), rdB = uint32_t((G::WM + wc + fr) * k8Row + sw);
    __syncthreads();

    // The per-lane offsets pass through empty asm statements where they are
    // used, so that addresses are formed there from uniform bases (kept in
    // scalar registers) instead of being kept per lane across the loop.
    auto fetch = [&](const int8_t* tA, const int8_t* tB, int chunk, int buf) {
        uint32_t vo = voff;
        __asm__ volatile("" : "+v"(vo));
        const uint64_t co = uint64_t(chunk) * 64;
#pragma unroll
        for (int i = 0; i < G::LOADS; ++i) {
            const int r0 = G::GROUP * i;  // first stage row of instruction i (all A or all B)
            const int8_t* base = (r0 < G::WM ? tA + uint64_t(r0) * rowBytes : tB + uint64_t(r0 - G::WM) * rowBytes) + co;
            __builtin_amdgcn_global_load_lds(base + vo, (lds_ptr_t)(lds + buf * G::BUF + w * 1024 + i * (G::NW * 1024)),
                                             16, 0, 0);
        }
    };
    v4i fa[RA], b0[CB], b1[CB];
    auto read_stage_b = [&](int buf, v4i(&b)[CB]) {
        uint32_t o = rdB;
        __asm__ volatile("" : "+v"(o));
        const uint8_t* p = lds + o + buf * G::BUF;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) b[cb] = *reinterpret_cast<const v4i*>(p + cb * 16 * k8Row);
    };
    auto a_row = [&](int buf) {
        uint32_t o = rdA;
        __asm__ volatile("" : "+v"(o));
        return lds + o + buf * G::BUF;
    };

    uint32_t tile = blockIdx.x, ta, tb;
    tile_coords_lg(tile, lgA, lgB, ta, tb);
    const int8_t* tA = A + uint64_t(ta) * G::WM * rowBytes;
    const int8_t* tB = B + uint64_t(tb) * G::WN * rowBytes;
#pragma unroll
    for (int c = 0; c < NBUF; ++c) fetch(tA, tB, kc0 + c, c);

    for (;;) {
        v4i acc[RA][CB];
#pragma unroll
        for (int i = 0; i < RA; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[i][j] = v4i{0, 0, 0, 0};
        // every load and store of the wave has completed (loads and stores
        // share one counter); stage 0 is visible to all waves. A fragments:
        // one set, each refilled with the next stage's as soon as its last
        // product of the stage is issued; B fragments: two sets
        chunk_barrier<0>();
        {
            const uint8_t* pa = a_row(0);
#pragma unroll
            for (int rb = 0; rb < RA; ++rb) fa[rb] = *reinterpret_cast<const v4i*>(pa + rb * 16 * k8Row);
        }
        read_stage_b(0, b0);

        const uint32_t next = tile + gridDim.x;
        const bool more = next < T;
        uint32_t nta = 0, ntb = 0;
        if (more) tile_coords_lg(next, lgA, lgB, nta, ntb);
        const int8_t* nA = A + uint64_t(nta) * G::WM * rowBytes;
        const int8_t* nB = B + uint64_t(ntb) * G::WN * rowBytes;
        // Stage kc from fa and bc. Other than the tile's last stage (LAST),
        // a step first waits until stage kc + 1 has landed with at most VM
        // loads (stages kc + 2, kc + 3) still in flight, so that no wave reads
        // stage kc any more; with FETCH its buffer then takes stage kc + 4;
        // stage kc + 1 is read into fa and bn.
        auto step = [&](int kc, v4i(&bc)[CB], v4i(&bn)[CB], auto vm, auto fetch_next, auto last) {
            constexpr int VM = decltype(vm)::value;
            constexpr bool FETCH = decltype(fetch_next)::value, LAST = decltype(last)::value;
            const uint8_t* pa = nullptr;
            if constexpr (!LAST) {
                chunk_barrier<VM>();
                if constexpr (FETCH) fetch(tA, tB, kc0 + kc + 4, kc & 3);
                // (the compiler would otherwise wait at the MFMAs for the
                // fragment reads below, to order them after the loads above)
                __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(63));
                read_stage_b((kc + 1) & 3, bn);
                pa = a_row((kc + 1) & 3);
            } else {
                // every fragment of the tile is in registers, so the four
                // buffers take the next tile's first stages
                chunk_barrier<63>();
                if (more)
#pragma unroll
                    for (int c = 0; c < NBUF; ++c) fetch(nA, nB, kc0 + c, c);
            }
#pragma unroll
            for (int rb = 0; rb < RA; ++rb) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[rb], bc[cb], acc[rb][cb], 0, 0, 0);
                if constexpr (!LAST) fa[rb] = *reinterpret_cast<const v4i*>(pa + rb * 16 * k8Row);
            }
        };
        using yes = std::true_type;
        using no = std::false_type;
        using vm2 = std::integral_constant<int, 2 * G::LOADS>;
        using vm1 = std::integral_constant<int, G::LOADS>;
        using vm0 = std::integral_constant<int, 0>;
        // Main loop: every step waits for the same count and fetches. The
        // sums stay exact in int32 for k8Flush stages; after each full range
        // they are reduced to centred residues (the last range ends in the
        // epilogue).
        int kc = 0;
        while (NK >= 4 && kc + 4 < nk) {
            const int end = std::min(nk - 4, kc + k8Flush);
            for (; kc < end; kc += 2) {
                step(kc, b0, b1, vm2(), yes(), no());
                step(kc + 1, b1, b0, vm2(), yes(), no());
            }
            if (kc < nk - 4) {
#pragma unroll
                for (int i = 0; i < RA; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[i][j][v] = ms.center32(acc[i][j][v]);
            }
        }
        // the last stages
        if constexpr (NK >= 4) {
            step(nk - 4, b0, b1, vm2(), no(), no());
            step(nk - 3, b1, b0, vm1(), no(), no());
            step(nk - 2, b0, b1, vm0(), no(), no());
            step(nk - 1, b1, b0, vm0(), no(), yes());
        } else if constexpr (NK == 2) {
            step(0, b0, b1, vm0(), no(), no());
            step(1, b1, b0, vm0(), no(), yes());
        } else {
            step(0, b0, b1, vm0(), no(), yes());
        }

        // epilogue: lane holds A index wr + 16 rb + 4 q + v, B index
        // wc + 16 cb + fr of each 16x16 block
        const int32_t negm = -int32_t(ms.m);
        const int32_t r16 = int32_t(ms.r16);
        auto packed = [&](int rb, int cb) {
            return pack4(res8<FOLD>(acc[rb][cb][0], r16, negm, ms.inv), res8<FOLD>(acc[rb][cb][1], r16, negm, ms.inv),
                         res8<FOLD>(acc[rb][cb][2], r16, negm, ms.inv), res8<FOLD>(acc[rb][cb][3], r16, negm, ms.inv));
        };
        if (splits > 1) {
            // partial residues of this K range, tile-local order (j, i): the
            // lane's four A indices are consecutive bytes
            int8_t* pt = part + blockIdx.z * part_stride + (uint64_t(blockIdx.y) * T + tile) * (G::WM * G::WN);
            uint32_t lo = uint32_t((wc + fr) * G::WM + wr + 4 * q);
            __asm__ volatile("" : "+v"(lo));
#pragma unroll
            for (int rb = 0; rb < RA; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    *reinterpret_cast<uint32_t*>(pt + lo + uint32_t(16 * cb * G::WM + 16 * rb)) = packed(rb, cb);
        } else {
            int ci = tid;
            __asm__ volatile("" : "+v"(ci));  // read here, per tile
            const uint64_t baseC =
                (pdep64(uint64_t(ta) * G::WM, a.maskA) | pdep64(uint64_t(tb) * G::WN, a.maskB)) | lconst[ci];
            store_tile8<RA, CB, FOLD>(acc, C, baseC, ex, ms, lane);
        }
        if (!more) break;
        tile = next;
        ta = nta;
        tb = ntb;
        tA = nA;
        tB = nB;
    }
}

// split-K: sum the partial residues of every K range and scatter into C
template <class G>
__global__ __launch_bounds__(256) void k_mfma8_reduce(StepArgs a, const int8_t* part, int64_t part_stride,
                                                      int splits) {
    const int g = blockIdx.z;
    const ModSmall ms{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};
    int8_t* C = static_cast<int8_t*>(a.C) + g * a.strideC;
    const int lgA = a.fA - G::LGM, lgB = a.fB - G::LGN;
    const uint64_t T = uint64_t(1) << (lgA + lgB);
    const uint64_t n = T * (G::WM * G::WN);
    const int8_t* pg = part + g * part_stride;
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t tile = e / (G::WM * G::WN), loc = e % (G::WM * G::WN);  // loc = j WM + i
        int32_t sum = 0;  // at most 1024 residues of magnitude 127
        for (int y = 0; y < splits; ++y) sum += pg[(uint64_t(y) * T + tile) * (G::WM * G::WN) + loc];
        uint32_t ta, tb;
        tile_coords_lg(uint32_t(tile), lgA, lgB, ta, tb);
        const uint64_t j = loc / G::WM, i = loc % G::WM;
        C[pdep64(uint64_t(ta) * G::WM + i, a.maskA) | pdep64(uint64_t(tb) * G::WN + j, a.maskB)] =
            int8_t(ms.center32(sum));
    }
}

// Short shared dimension, K = 2^S <= 32: no staging. Each lane reads its
// fragments straight from A's and B's rows (K consecutive bytes, the tile's
// rows consecutive in memory, so a wave's fragment load covers 16 whole rows)
// -- 8 bytes at K offset 8 q, zero where 8 q >= K -- and one
// v_mfma_i32_16x16x32_i8 per 16x16 block gives the exact sums (at most
// 32 127^2 < 2^21). Such steps are bound by writing C. A wave takes U tiles
// per round: their fragments are requested together (each set as soon as its
// tile's products are issued) and one wait per round covers them. (Loads and
// stores share one completion counter, so that wait also covers the stores
// before it; measured on the largest 1-in-3 configuration, U = 2 and 4 are no
// faster than U = 1.)
template <class G, int S, int U = 1>
__global__ __launch_bounds__(G::THREADS) void k_mfma8_short(StepArgs a, Mfma8Extra ex) {
    constexpr int RA = G::RA, CB = G::CB, K = 1 << S;
    const int g = blockIdx.z;
    const int8_t* A = static_cast<const int8_t*>(a.A) + g * a.strideA;
    const int8_t* B = static_cast<const int8_t*>(a.B) + g * a.strideB;
    int8_t* C = static_cast<int8_t*>(a.C) + g * a.strideC;
    const ModSmall ms{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (w % G::WAVES_A) * 16 * RA, wc = (w / G::WAVES_A) * 16 * CB;
    const int lgA = a.fA - G::LGM, lgB = a.fB - G::LGN;
    const uint32_t T = 1u << (lgA + lgB);
    const int fr = lane & 15, q = lane >> 4;
    const uint64_t lc = lane_offset8<RA>(a, ex, wr, wc, lane);
    // lane's fragment offset within a tile's rows: row wr + fr (A) or
    // wc + fr (B), K offset 8 q
    const uint32_t offA = uint32_t((wr + fr) * K + 8 * q), offB = uint32_t((wc + fr) * K + 8 * q);
    typedef long frag_t;
    auto load = [&](const int8_t* p) -> frag_t {
        if constexpr (S >= 3) {
            if (8 * q >= K) return 0;
            return *reinterpret_cast<const frag_t*>(p);
        } else {
            if (q != 0) return 0;
            if constexpr (S == 2) return frag_t(*reinterpret_cast<const uint32_t*>(p));
            if constexpr (S == 1) return frag_t(*reinterpret_cast<const uint16_t*>(p));
            return frag_t(*reinterpret_cast<const uint8_t*>(p));
        }
    };
    frag_t fa[U][RA], fb[U][CB];
    auto fetch = [&](uint32_t tile, int u) {
        uint32_t ta, tb;
        tile_coords_lg(tile, lgA, lgB, ta, tb);
        const int8_t* pA = A + uint64_t(ta) * G::WM * K + offA;
        const int8_t* pB = B + uint64_t(tb) * G::WN * K + offB;
#pragma unroll
        for (int rb = 0; rb < RA; ++rb) fa[u][rb] = load(pA + 16 * K * rb);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) fb[u][cb] = load(pB + 16 * K * cb);
    };
    const uint32_t stride = gridDim.x;
    uint32_t tile = blockIdx.x;
    if (tile >= T) return;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (tile + u * stride < T) fetch(tile + u * stride, u);
    for (;;) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t t = tile + u * stride;
            if (t >= T) break;
            v4i acc[RA][CB];
#pragma unroll
            for (int rb = 0; rb < RA; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_i32_16x16x32_i8(fa[u][rb], fb[u][cb], v4i{0, 0, 0, 0}, 0, 0, 0);
            const uint32_t next = t + U * stride;
            if (next < T) fetch(next, u);
            uint32_t ta, tb;
            tile_coords_lg(t, lgA, lgB, ta, tb);
            const uint64_t baseC = (pdep64(uint64_t(ta) * G::WM, a.maskA) | pdep64(uint64_t(tb) * G::WN, a.maskB)) | lc;
            store_tile8<RA, CB, false>(acc, C, baseC, ex, ms, lane);
        }
        tile += U * stride;
        if (tile >= T) break;
    }
}

uint64_t pdep_host(uint64_t x, uint64_t m) {
    uint64_t r = 0;
    for (; m; m &= m - 1, x >>= 1)
        if (x & 1) r |= m & (~m + 1);
    return r;
}

Mfma8Extra extra_of(const StepArgs& a) {
    Mfma8Extra ex{};
    for (int rb = 0; rb < 8; ++rb) ex.dA[rb] = pdep_host(uint64_t(16 * rb), a.maskA);
    for (int v = 0; v < 4; ++v) ex.dV[v] = pdep_host(uint64_t(v), a.maskA);
    for (int cb = 0; cb < 4; ++cb) ex.dB[cb] = pdep_host(uint64_t(16 * cb), a.maskB);
    // v_perm selectors: bytes 0..3 of the neighbour's word are 0..3, the
    // lane's own are 4..7
    if ((a.maskA & 3) == 3) {
        ex.mode = 0;
        ex.sel[0] = ex.sel[1] = 0x07060504u;
    } else if ((a.maskB & 1) && (a.maskA & 2)) {  // C bit 0 from B, bit 1 from A
        ex.mode = 1;
        ex.sel[0] = 0x01050004u;  // own v0, neighbour v0, own v1, neighbour v1
        ex.sel[1] = 0x07030602u;  // neighbour v2, own v2, neighbour v3, own v3
    } else if ((a.maskA & 1) && (a.maskB & 2)) {  // C bit 0 from A, bit 1 from B
        ex.mode = 1;
        ex.sel[0] = 0x01000504u;  // own v0, own v1, neighbour v0, neighbour v1
        ex.sel[1] = 0x07060302u;  // neighbour v2, neighbour v3, own v2, own v3
    } else {
        ex.mode = 2;
    }
    // lane bit holding C bit pos (modes 0 and 1), -1 if none
    auto lane_bit_of = [&](int pos) -> int {
        const bool fromA = (a.maskA >> pos) & 1;
        const int idx = __builtin_popcountll((fromA ? a.maskA : a.maskB) & ((uint64_t(1) << pos) - 1));
        if (fromA) {
            if (idx == 2 || idx == 3) return 4 + (idx - 2);
            return idx == 1 && ex.mode == 1 ? 0 : -1;
        }
        if (idx >= 1 && idx <= 3) return idx;
        return idx == 0 && ex.mode == 0 ? 0 : -1;
    };
    ex.x2 = ex.x3 = -1;
    if (ex.mode != 2) {
        const int b2 = lane_bit_of(2), b3 = lane_bit_of(3);
        if (b2 >= 0 && b3 >= 0 && b2 != b3) {
            ex.x2 = b2;
            ex.x3 = b3;
        }
    }
    // the compiled 16-byte variants: (pair exchange, lane bit of C bit 2, of
    // C bit 3) with bits 4 and 5 by permlane swaps and 0..3 at run time
    const int c2 = ex.x2 >= 4 ? ex.x2 : 0, c3 = ex.x3 >= 4 ? ex.x3 : 0;
    ex.form = 0;
    if (ex.x2 >= 0) {
        if (ex.mode == 0 && c2 == 4 && c3 == 5) ex.form = 1;
        else if (ex.mode == 0 && c2 == 4 && c3 == 0) ex.form = 2;
        else if (ex.mode == 0 && c2 == 0 && c3 == 4) ex.form = 3;
        else if (ex.mode == 0 && c2 == 0 && c3 == 0) ex.form = 4;
        else if (ex.mode == 1 && c2 == 0 && c3 == 4) ex.form = 5;
        else if (ex.mode == 1 && c2 == 0 && c3 == 0) ex.form = 6;
    }
    if (ex.form == 0) ex.x2 = ex.x3 = -1;  // the lane offsets of 4-byte stores
    return ex;
}

template <class Gm>
hipError_t launch_cfg(const StepArgs& a, int G, hipStream_t stream, char* scratch, int64_t scratch_per_plane) {
    const Mfma8Extra ex = extra_of(a);
    const uint64_t T = (uint64_t(1) << (a.fA - Gm::LGM)) * (uint64_t(1) << (a.fB - Gm::LGN));
    // too few output tiles to fill the GPU: split K over block rows (powers
    // of two, as many partial tiles per plane as the scratch area holds, at
    // least 8 stages each so that reading operands outweighs writing the
    // partial tile)
    const int nk = 1 << (a.s - 6);
    const uint64_t cap_tiles = uint64_t(scratch_per_plane) / uint64_t(Gm::WM * Gm::WN);
    int splits = 1;
    while (T * G * splits * 2 <= 1024 && splits * 16 <= nk && T * splits * 2 <= cap_tiles) splits *= 2;
    int8_t* part = reinterpret_cast<int8_t*>(scratch);
    dim3 grid(uint32_t(std::min<uint64_t>(T, 1024)), uint32_t(splits), G);
    const int per = nk / splits;
    // sums of at most 8 stages stay below 8 64 127^2 < 2^23: no fold
    if (per > 8)
        hipLaunchKernelGGL((k_mfma8<Gm, 4, true>), grid, dim3(Gm::THREADS), 0, stream, a, ex, splits, part,
                           scratch_per_plane);
    else if (per >= 4)
        hipLaunchKernelGGL((k_mfma8<Gm, 4, false>), grid, dim3(Gm::THREADS), 0, stream, a, ex, splits, part,
                           scratch_per_plane);
    else if (per == 2)
        hipLaunchKernelGGL((k_mfma8<Gm, 2, false>), grid, dim3(Gm::THREADS), 0, stream, a, ex, splits, part,
                           scratch_per_plane);
    else
        hipLaunchKernelGGL((k_mfma8<Gm, 1, false>), grid, dim3(Gm::THREADS), 0, stream, a, ex, splits, part,
                           scratch_per_plane);
    if (splits > 1) {
        const uint64_t n = T * uint64_t(Gm::WM * Gm::WN);
        dim3 gr(uint32_t(std::min<uint64_t>((n + 255) / 256, 4096)), 1, G);
        hipLaunchKernelGGL((k_mfma8_reduce<Gm>), gr, dim3(256), 0, stream, a, part, scratch_per_plane, splits);
    }
    return hipGetLastError();
}

template <class Gm, int S>
hipError_t launch_short(const StepArgs& a, int G, hipStream_t stream) {
    const uint64_t T = (uint64_t(1) << (a.fA - Gm::LGM)) * (uint64_t(1) << (a.fB - Gm::LGN));
    dim3 grid(uint32_t(std::min<uint64_t>(T, 2048)), 1, G);
    hipLaunchKernelGGL((k_mfma8_short<Gm, S>), grid, dim3(Gm::THREADS), 0, stream, a, extra_of(a));
    return hipGetLastError();
}

template <class Gm>
hipError_t launch_short_s(const StepArgs& a, int G, hipStream_t stream) {
    switch (a.s) {
        case 0: return launch_short<Gm, 0>(a, G, stream);
        case 1: return launch_short<Gm, 1>(a, G, stream);
        case 2: return launch_short<Gm, 2>(a, G, stream);
        case 3: return launch_short<Gm, 3>(a, G, stream);
        case 4: return launch_short<Gm, 4>(a, G, stream);
        default: return launch_short<Gm, 5>(a, G, stream);
    }
}

}  // namespace

bool mfma8_eligible(const StepArgs& a) {
    // at least one 128 x 64 tile, K of at least one 64-entry chunk, a
    // stage's rows within 32-bit load offsets and the tile count in 32 bits
    // (K below 64: the unstaged kernel, 128 x 128 or 128 x 64 tiles)
    return a.s >= 0 && a.s <= k8MaxRowBytesLog && a.fA >= 7 && a.fB >= 6 && a.fA + a.fB <= 45;
}

// The tile shape of the built-in rule: the largest that fits both free sides.
int mfma8_rule_cfg(const StepArgs& a) {
    if (a.fB >= 8) return MFMA8_256x256;
    if (a.fB == 7) return a.fA >= 8 ? MFMA8_256x128 : MFMA8_128x128;
    return a.fA >= 8 ? MFMA8_256x64 : MFMA8_128x64;
}

hipError_t launch_mfma8_cfg(const StepArgs& a, int G, hipStream_t stream, char* scratch, int64_t scratch_per_plane,
                            int cfg) {
    if (!mfma8_eligible(a) || (cfg != MFMA8_RULE && !mfma8_cfg_fits(cfg, a.fA, a.fB))) return hipErrorInvalidValue;
    if (a.s < 6)
        return a.fB >= 7 ? launch_short_s<Cfg128x128>(a, G, stream) : launch_short_s<Cfg128x64>(a, G, stream);
    if (cfg == MFMA8_RULE) cfg = mfma8_rule_cfg(a);
    switch (cfg) {
        case MFMA8_256x256: return launch_cfg<Cfg256x256>(a, G, stream, scratch, scratch_per_plane);
        case MFMA8_256x128: return launch_cfg<Cfg256x128>(a, G, stream, scratch, scratch_per_plane);
        case MFMA8_128x128: return launch_cfg<Cfg128x128>(a, G, stream, scratch, scratch_per_plane);
        case MFMA8_256x64: return launch_cfg<Cfg256x64>(a, G, stream, scratch, scratch_per_plane);
        default: return launch_cfg<Cfg128x64>(a, G, stream, scratch, scratch_per_plane);
    }
}

hipError_t launch_mfma8(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                        double step_macs, char* scratch, int64_t scratch_per_plane) {
    if (!mfma8_eligible(a)) return hipErrorInvalidValue;
    prof->before(stream);
    // the autotuner's measured tile shape for the nearest tuned shape, else the rule
    const int cfg = a.s >= 6 ? tuned_choice(TK_MFMA8, EL_I8, a.fA, a.fB, a.s) : MFMA8_RULE;
    const hipError_t e = launch_mfma8_cfg(a, G, stream, scratch, scratch_per_plane, cfg);
    prof->after_raw(stream, KC_MFMA, step_bytes, step_macs);
    return e;
}

}  // namespace tn
