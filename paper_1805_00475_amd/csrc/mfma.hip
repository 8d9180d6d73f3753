// Dense contraction steps on the matrix cores, exactly.
//
// A step whose shared dimension K = 2^s is wide and whose two free sides are
// large is a plain matrix product C = A B^T over residues modulo p < 65280
// (rows of A and B are contiguous along the shared bonds in the plan's
// layout). Each residue r is centred to r' in (-p/2, p/2] (|r'| <= 32639) and
// written as two signed base-256 digits r' = d0 + d1 2^8, d0 and d1 in
// [-128, 127]. Then
//     C = T0 + 2^8 T1 + 2^16 T2,   T_t = sum_{i+j=t} A_i B_j^T,
// where A_i, B_j are int8 digit matrices; every T_t is accumulated by the
// int8 MFMA into int32 registers. Each product of digits is at most 2^14 in
// magnitude and at most two digit pairs share a shift, so K <= 2^15 keeps
// every T_t at most 2^30 -- exact; wider K is summed in ranges of 2^15, each
// reduced to a residue that seeds the next range. The epilogue forms
// X = T0 + 2^8 T1 + 2^16 T2 (|X| < 2^47) and reduces it modulo p in double
// precision, where every step is exact.
//
// Two kernels per step: k_digits rewrites A and B in place (they die at this
// step) so that every 64-entry chunk of a row (256 bytes) starts with its two
// digit planes of 64 bytes each; k_mfma then copies digit tiles into LDS and
// runs v_mfma_i32_16x16x64_i8. Output tiles are staged in LDS and written in
// C-address order so stores stay coalesced for any bit interleaving.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "mfma.hpp"
#include "mfma_common.hpp"
#include "profile.hpp"

namespace tn {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- digit pass
constexpr int kDigits = 2;
// Digit planes of four consecutive residues: word d holds digit d of each
// (byte k = residue k). In a digit-plane tensor, entry e's digit d is byte
// 256 (e / 64) + 64 d + e % 64 (bytes 128..255 of every 64-entry chunk are
// unused), so the word of entries 4m..4m+3 (m = e / 4) of plane d sits at
// word 64 (e / 64) + 16 d + (e % 64) / 4.
__device__ __forceinline__ void digit_words(const uint32_t (&r)[4], uint32_t p, uint32_t (&w)[kDigits]) {
    const uint32_t half = p >> 1;
    w[0] = w[1] = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t c = r[e] > half ? int32_t(r[e] - p) : int32_t(r[e]);
        const int32_t d0 = int32_t(int8_t(c & 0xff));
        const int32_t d1 = (c - d0) >> 8;  // in [-128, 127] since |c| <= 32639
        w[0] |= (uint32_t(d0) & 0xffu) << (8 * e);
        w[1] |= (uint32_t(d1) & 0xffu) << (8 * e);
    }
}

// In place: the 16 lanes owning one 64-entry chunk read it (4 entries each)
// before any of them writes, since they are consecutive lanes of one wave
// and every store depends on all four loads of that lane.
__global__ __launch_bounds__(256) void k_digits(uint32_t* X, int64_t stride, uint64_t n_vec4,
                                                StepArgs a) {
    const uint32_t p = a.p[blockIdx.z];
    uint32_t* base = X + blockIdx.z * stride;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n_vec4;
         v += uint64_t(gridDim.x) * blockDim.x) {
        uint4 r = reinterpret_cast<const uint4*>(base)[v];
        const uint32_t rv[4] = {r.x, r.y, r.z, r.w};
        uint32_t w[kDigits];
        digit_words(rv, p, w);
        // chunk = 16 vec4 of 64 entries; plane d of the chunk at byte 64 d
        const uint64_t chunk = v >> 4;
        const uint32_t lane16 = uint32_t(v & 15);
        uint32_t* cbase = base + chunk * 64;
#pragma unroll
        for (int d = 0; d < kDigits; ++d) cbase[d * 16 + lane16] = w[d];
    }
}

// --------------------------------------------------------------- GEMM
// Work-group tile 128 (xA) x 64 (xB), used when B's free side has 6 bits.
// Each launch row sums at most 2^15 entries of K (one exact range; wider K
// is always split over block rows). 8 waves of 32 x 32 (two per SIMD), K
// consumed in stages of 128 entries: the two digit planes of two 64-entry
// chunks (one 16x16x64 MFMA per chunk, digit pair and 16x16 block, 16 per
// wave and chunk). Digit tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: one wave instruction fills 1 KiB, four 256-byte
// rows) through three buffers; stage k+3 is requested while stage k is
// multiplied, two stages before it is read, since every stage is first read
// by one of the work-groups sharing it, which waits for HBM or the last-level
// cache. The barrier that makes stage k+1 visible sits between the two
// chunks of stage k: the fragments of stage k's second chunk are read while
// its first chunk is multiplied, and those of stage k+1's first chunk while
// its second chunk is, so the matrix cores do not wait for LDS reads after a
// barrier. The next tile's first two stages are requested at the last
// barrier of the current tile, before its last chunk and epilogue. When
// K = 64 a stage holds one chunk (loaded twice, multiplied once).
//
// LDS rows are 256 bytes (one stage of one row, 16 slots of 16 bytes; slot
// 8 h + 4 d + q = bytes 16 q.. of plane d of chunk h) with slot c of row r
// stored at slot c ^ (r % 16). A fragment read has the 16 lanes of a
// quarter-wave on 16 consecutive rows at one logical slot, so the XOR spreads
// them over all 16 slots (all 64 banks): conflict-free. Plain rows would put
// them on one slot.
constexpr int kBM = 128, kBN = 64, kRowB = 256;  // LDS row stride (bytes)
constexpr int kBuf = (kBM + kBN) * kRowB;        // one LDS buffer (48 KiB)
constexpr int kStages = 3;
constexpr int kThreads = 512;

// X = T0 + 2^8 T1 + 2^16 T2 with every |T_t| <= 2^30 is an integer below
// 2^47 in magnitude, so double precision holds it and every step below
// exactly: X itself (two fused multiply-adds), q = floor(X inv_p) with
// inv_p the double nearest 1/p (off from floor(X / p) by at most one, as
// X / p < 2^32 and the product's error is below 2^-20), and X - q p (below
// 2p in magnitude, one fused multiply-add). Two conditional corrections
// give X mod p. Double-precision operations run at the full vector rate,
// which makes this cheaper than 64-bit integer folds.
constexpr int kShifts = 2 * kDigits - 1;
__device__ __forceinline__ uint32_t combine_digits(const int32_t (&T)[kShifts], uint32_t p, double inv_p) {
    const double x = fma(double(T[2]), 65536.0, fma(double(T[1]), 256.0, double(T[0])));
    const double pd = double(p);
    const double q = floor(x * inv_p);
    int32_t r = int32_t(fma(-q, pd, x));
    r += r < 0 ? int32_t(p) : 0;
    r -= r >= int32_t(p) ? int32_t(p) : 0;
    return uint32_t(r);
}


// Every 2^15 entries of K the exact sums are reduced: T0 takes the residue
// of X (below p < 2^16) and T1, T2 restart from zero, so the next range adds
// at most 2^29 to T0 and the bounds above hold again.
template <int RB, int CB>
__device__ __forceinline__ void flush(v4i (&acc)[kShifts][RB][CB], uint32_t p, double inv_p) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int32_t Tt[kShifts];
#pragma unroll
                for (int t = 0; t < kShifts; ++t) Tt[t] = acc[t][rb][cb][v];
                acc[0][rb][cb][v] = int32_t(combine_digits(Tt, p, inv_p));
#pragma unroll
                for (int t = 1; t < kShifts; ++t) acc[t][rb][cb][v] = 0;
            }
}

// One stage of a tile into LDS buffer `dst` (wave's 1 KiB slice): A rows
// 4 (w + 8 i) + lane / 16 for i < 4, B rows 4 (w + 8 i) + lane / 16 for i < 2.
__device__ __forceinline__ void fetch_chunk(const uint8_t* gA, const uint8_t* gB, uint64_t rows32, uint8_t* dst) {
    __builtin_amdgcn_global_load_lds(gA, (lds_ptr_t)dst, 16, 0, 0);
    __builtin_amdgcn_global_load_lds(gA + rows32, (lds_ptr_t)(dst + 8 * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(gA + 2 * rows32, (lds_ptr_t)(dst + 16 * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(gA + 3 * rows32, (lds_ptr_t)(dst + 24 * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(gB, (lds_ptr_t)(dst + kBM * kRowB), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(gB + rows32, (lds_ptr_t)(dst + kBM * kRowB + 8 * 1024), 16, 0, 0);
}
constexpr int kLoadsPerChunk = 6;

// Fragments of chunk h of the stage in LDS buffer `src`: A rows wr + fr
// (+16) and B rows wc + fr (+16) at the wave's logical slot of each digit.
struct Frags {
    v4i a[kDigits][2], b[kDigits][2];
};
__device__ __forceinline__ void read_frags(const uint8_t* src, int wr, int wc, int fr,
                                           const int (&sw)[kDigits], Frags& f) {
    const uint8_t* rA = src + (wr + fr) * kRowB;
    const uint8_t* rB = src + (kBM + wc + fr) * kRowB;
    auto ld = [](const uint8_t* q) { return *reinterpret_cast<const v4i*>(q); };
#pragma unroll
    for (int d = 0; d < kDigits; ++d) {
        f.a[d][0] = ld(rA + sw[d]);
        f.a[d][1] = ld(rA + 16 * kRowB + sw[d]);
        f.b[d][0] = ld(rB + sw[d]);
        f.b[d][1] = ld(rB + 16 * kRowB + sw[d]);
    }
}

// 16 MFMAs of one chunk: digit pair (i, j) of every 16x16 block pair into
// shift group i + j.
__device__ __forceinline__ void mfma_chunk(const Frags& f, v4i (&acc)[kShifts][2][2]) {
#pragma unroll
    for (int i = 0; i < kDigits; ++i)
#pragma unroll
        for (int j = 0; j < kDigits; ++j)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    acc[i + j][rb][cb] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8(f.a[i][rb], f.b[j][cb], acc[i + j][rb][cb], 0, 0, 0);
}

// TWO: K >= 128 (two chunks per stage); otherwise K = 64 (one chunk).
template <bool TWO>
__global__ __launch_bounds__(kThreads, 1) void k_mfma(StepArgs a, MfmaExtra ex, int splits, uint32_t* part,
                                                      int64_t part_stride) {
    __shared__ __align__(1024) uint8_t lds[kStages * kBuf];
    // output staging (kBM x kBN words) lives in the third buffer, so the next
    // tile's first two chunks can load into the other two meanwhile
    uint32_t* sOut = reinterpret_cast<uint32_t*>(lds + 2 * kBuf);

    const int g = blockIdx.z;
    const uint8_t* A = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.A) + g * a.strideA);
    const uint8_t* B = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.B) + g * a.strideB);
    uint32_t* C = static_cast<uint32_t*>(a.C) + g * a.strideC;
    const uint32_t p = a.p[g];
    const double inv_p = ex.inv_p[g];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: LDS slice bases stay scalar
    const int wr = (w & 3) * 32, wc = (w >> 2) * 32;
    const uint64_t rowBytes = uint64_t(4) << a.s;  // K entries of 4 bytes (digit planes in the first half of each chunk)
    const int nk_all = TWO ? 1 << (a.s - 7) : 1;  // stages of 128 entries
    // split-K: block row blockIdx.y owns stages [kc0, kc0 + nk)
    const int nk = nk_all / splits;
    const int kc0 = int(blockIdx.y) * nk;
    const uint64_t tilesA = uint64_t(1) << (a.fA - 7), tilesB = uint64_t(1) << (a.fB - 6);
    const uint64_t T = tilesA * tilesB;
    if (uint64_t(blockIdx.x) >= T) return;  // whole work-group

    // output mapping inside a tile: tile-local t = 4 tid + k + 2048 q (k, q < 4)
    // at position pdep(t, TM), TM = the 7 lowest A bits and 6 lowest B bits
    // of C. The 6 lowest bits of C are always tile bits (at most 6 of them
    // come from either side), so k adds to the position: each thread writes
    // four consecutive words, one 16-byte store per q.
    const uint64_t TM = pdep64(127, a.maskA) | pdep64(63, a.maskB);
    const uint64_t offLow = pdep64(uint64_t(4 * tid), TM);
    const uint32_t iLow = uint32_t(pext64(offLow, a.maskA)), jLow = uint32_t(pext64(offLow, a.maskB));
    // loads: lane l of wave w brings row ldRow = 4 w + l / 16 (+ 32 i) into
    // physical slot l % 16, i.e. logical slot c = (l % 16) ^ (ldRow % 16):
    // bytes 16 (c % 8).. of chunk c / 8 of the stage (chunk 0 when K = 64);
    // stage k starts at byte 512 k of the row
    const int ldRow = 4 * w + (lane >> 4);
    const int ldSlot = (lane & 15) ^ (ldRow & 15);
    const uint64_t ldOff = uint64_t(ldRow) * rowBytes + uint64_t(TWO ? (ldSlot >> 3) * 256 : 0) +
                           uint64_t((ldSlot & 7) * 16);
    const uint64_t rows32 = 32 * rowBytes;
    uint8_t* const ldsW = lds + w * 1024;
    const int fr = lane & 15;
    // fragment of digit d of chunk h: logical slot 8 h + 4 d + lane / 16 of
    // row (.. + fr)
    const int q4 = (lane >> 4) ^ fr;
    const int sw[2][kDigits] = {{q4 * 16, (q4 ^ 4) * 16}, {(q4 ^ 8) * 16, (q4 ^ 12) * 16}};
    __syncthreads();

    uint64_t tile = blockIdx.x, ta, tb;
    tile_coords(tile, tilesA, tilesB, ta, tb);
    const uint8_t* gA = A + ta * kBM * rowBytes + ldOff;
    const uint8_t* gB = B + tb * kBN * rowBytes + ldOff;
    fetch_chunk(gA + uint64_t(kc0) * 512, gB + uint64_t(kc0) * 512, rows32, ldsW);
    if (nk > 1) fetch_chunk(gA + uint64_t(kc0 + 1) * 512, gB + uint64_t(kc0 + 1) * 512, rows32, ldsW + kBuf);

    for (;;) {
        v4i acc[kShifts][2][2];
#pragma unroll
        for (int t = 0; t < kShifts; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[t][i][j] = v4i{0, 0, 0, 0};

        // stage 0 has landed (stage 1 may still be in flight), and every
        // wave is done with the previous tile's output staging in buffer 2
        if (nk > 1)
            chunk_barrier<kLoadsPerChunk>();
        else
            chunk_barrier<0>();
        if (nk > 2) fetch_chunk(gA + uint64_t(kc0 + 2) * 512, gB + uint64_t(kc0 + 2) * 512, rows32, ldsW + 2 * kBuf);
        Frags f0, f1;
        read_frags(lds, wr, wc, fr, sw[0], f0);

        const uint64_t next = tile + gridDim.x;
        const bool more = next < T;
        uint64_t nta = 0, ntb = 0;
        const uint8_t *nA = gA, *nB = gB;
        int buf = 0;  // kc % 3
        for (int kc = 0; kc + 1 < nk; ++kc) {
            const int nb = buf == 2 ? 0 : buf + 1;
            read_frags(lds + buf * kBuf, wr, wc, fr, sw[1], f1);
            mfma_chunk(f0, acc);
            // stage kc + 1 has landed (kc + 2 may be in flight) and no wave
            // reads stage kc any more: its buffer takes stage kc + 3
            if (kc + 2 < nk)
                chunk_barrier<kLoadsPerChunk>();
            else
                chunk_barrier<0>();
            if (kc + 3 < nk)
                fetch_chunk(gA + uint64_t(kc0 + kc + 3) * 512, gB + uint64_t(kc0 + kc + 3) * 512, rows32,
                            ldsW + buf * kBuf);
            read_frags(lds + nb * kBuf, wr, wc, fr, sw[0], f0);
            mfma_chunk(f1, acc);
            buf = nb;
        }
        // last stage
        if (TWO) read_frags(lds + buf * kBuf, wr, wc, fr, sw[1], f1);
        mfma_chunk(f0, acc);
        // every fragment of this tile is in registers: buffers 0 and 1 take
        // the next tile's first stages, buffer 2 the output staging
        chunk_barrier<63>();
        if (more) {
            tile_coords(next, tilesA, tilesB, nta, ntb);
            nA = A + nta * kBM * rowBytes + ldOff;
            nB = B + ntb * kBN * rowBytes + ldOff;
            fetch_chunk(nA + uint64_t(kc0) * 512, nB + uint64_t(kc0) * 512, rows32, ldsW);
            if (nk > 1) fetch_chunk(nA + uint64_t(kc0 + 1) * 512, nB + uint64_t(kc0 + 1) * 512, rows32, ldsW + kBuf);
        }
        if (TWO) mfma_chunk(f1, acc);
        // epilogue: lane holds rows 4 (lane / 16) + v, column lane % 16 of each 16x16 block
        if (splits > 1) {
            // partial residue of this K range, tile-local order (i, j)
            uint32_t* pt = part + blockIdx.z * part_stride + (uint64_t(blockIdx.y) * T + tile) * (kBM * kBN);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int32_t Tt[kShifts];
#pragma unroll
                        for (int t = 0; t < kShifts; ++t) Tt[t] = acc[t][rb][cb][v];
                        const int i = wr + rb * 16 + 4 * (lane >> 4) + v;
                        const int j = wc + cb * 16 + fr;
                        pt[i * kBN + j] = combine_digits(Tt, p, inv_p);
                    }
        } else {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int32_t Tt[kShifts];
#pragma unroll
                        for (int t = 0; t < kShifts; ++t) Tt[t] = acc[t][rb][cb][v];
                        const int i = wr + rb * 16 + 4 * (lane >> 4) + v;
                        const int j = wc + cb * 16 + fr;
                        sOut[i * kBN + j] = combine_digits(Tt, p, inv_p);
                    }
            // staging complete (the next tile's loads may stay in flight)
            chunk_barrier<63>();
            const uint64_t baseC = pdep64(ta * kBM, a.maskA) | pdep64(tb * kBN, a.maskB);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t o = offLow | ex.hiOff[q];
                const uint32_t i = iLow | ex.hiI[q];
                const uint32_t j = jLow | ex.hiJ[q];
                const uint32_t v[4] = {sOut[i * kBN + j], sOut[(i | ex.dI[1]) * kBN + (j | ex.dJ[1])],
                                       sOut[(i | ex.dI[2]) * kBN + (j | ex.dJ[2])],
                                       sOut[(i | ex.dI[3]) * kBN + (j | ex.dJ[3])]};
                const uint64_t e = baseC | o;
                if (ex.digits_out) {
                    // the consumer is a matrix-core step: hand over digit planes
                    uint32_t w[kDigits];
                    digit_words(v, p, w);
                    uint32_t* cw = C + (e >> 6) * 64 + ((e & 63) >> 2);
#pragma unroll
                    for (int d = 0; d < kDigits; ++d) cw[16 * d] = w[d];
                } else {
                    *reinterpret_cast<uint4*>(C + e) = uint4{v[0], v[1], v[2], v[3]};
                }
            }
        }
        if (!more) break;
        tile = next;
        ta = nta;
        tb = ntb;
        gA = nA;
        gB = nB;
    }
}


// ------------------------------------------------------ square-tile GEMM
// Work-group tile 128 (xA) x 128 (xB), 8 waves of 64 x 32 (two per SIMD),
// used when both free sides have at least 7 bits. Per entry of K the tile
// loads 512 bytes of digits for 16384 outputs, a third less than the
// 128 x 64 tile above, and each wave reads 48 fragment registers per chunk
// for 32 MFMAs instead of 32 for 16: the loads into LDS, not the matrix
// cores, bound the narrower tile. K goes in stages of one 64-entry chunk
// (128-byte LDS rows: the two digit planes) through four 32 KiB buffers.
// Chunk k+4 is requested while chunk k is multiplied; one barrier per chunk
// makes chunk k+1 visible and frees chunk k's buffer, after which the wave
// reads chunk k+1's fragments while chunk k's MFMAs run (fragment register
// sets alternate between chunks). The next tile's first two chunks are
// requested at the tile's last barrier; the output staging (64 KiB) uses
// buffers 2 and 3.
//
// LDS rows are 128 bytes (8 slots of 16 bytes; slot 4 d + q = bytes 16 q..
// of plane d), slot c of row r stored at slot c ^ (r % 8). A 16-byte read is
// served eight lanes at a time, free of bank conflicts when they cover 128
// distinct bytes modulo 128; a fragment read has eight consecutive lanes on
// eight consecutive rows (128 bytes apart) at one logical slot, which the
// XOR sends to eight distinct slots.
constexpr int kSqM = 128, kSqN = 128, kSqRow = 128;
constexpr int kSqBuf = (kSqM + kSqN) * kSqRow;  // 32 KiB
constexpr int kSqBufs = 4;
constexpr int kSqLoads = 4;               // load instructions per wave and chunk
constexpr int kSqFlush = (1 << 15) / 64;  // chunks per exact int32 range

struct SqFrags {
    v4i a[kDigits][4], b[kDigits][2];
};

// fragments of the chunk in buffer `src`: A rows wr + 16 rb + fr, B rows
// wc + 16 cb + fr, each at the lane's slot of digit plane d
__device__ __forceinline__ void sq_read(const uint8_t* src, int wr, int wc, int fr, const int (&sw)[kDigits],
                                        SqFrags& f) {
    const uint8_t* rA = src + (wr + fr) * kSqRow;
    const uint8_t* rB = src + (kSqM + wc + fr) * kSqRow;
    auto ld = [](const uint8_t* q) { return *reinterpret_cast<const v4i*>(q); };
#pragma unroll
    for (int d = 0; d < kDigits; ++d) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) f.a[d][rb] = ld(rA + rb * 16 * kSqRow + sw[d]);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) f.b[d][cb] = ld(rB + cb * 16 * kSqRow + sw[d]);
    }
}

__device__ __forceinline__ void sq_mfma(const SqFrags& f, v4i (&acc)[kShifts][4][2]) {
#pragma unroll
    for (int i = 0; i < kDigits; ++i)
#pragma unroll
        for (int j = 0; j < kDigits; ++j)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    acc[i + j][rb][cb] =
                        __builtin_amdgcn_mfma_i32_16x16x64_i8(f.a[i][rb], f.b[j][cb], acc[i + j][rb][cb], 0, 0, 0);
}

// One chunk of a tile into LDS buffer `dst` (wave's 1 KiB slices): lane l
// of wave w brings tile row 8 w + l / 8 (+ 64) of A and of B, 16 bytes at
// byte voff of that row; tA, tB are the tiles' first rows (wave-uniform).
__device__ __forceinline__ void sq_fetch(const uint8_t* tA, const uint8_t* tB, uint64_t chunk, uint64_t rows64,
                                         uint32_t voff, uint8_t* dst) {
    const uint64_t co = chunk * 256;
    __builtin_amdgcn_global_load_lds(tA + co + voff, (lds_ptr_t)dst, 16, 0, 0);
    __builtin_amdgcn_global_load_lds(tA + co + rows64 + voff, (lds_ptr_t)(dst + 8 * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(tB + co + voff, (lds_ptr_t)(dst + 16 * 1024), 16, 0, 0);
    __builtin_amdgcn_global_load_lds(tB + co + rows64 + voff, (lds_ptr_t)(dst + 24 * 1024), 16, 0, 0);
}

__global__ __launch_bounds__(kThreads, 1) void k_mfma_sq(StepArgs a, MfmaExtra ex, int splits, uint32_t* part,
                                                         int64_t part_stride) {
    // chunk buffers, then per-thread epilogue constants: kept in LDS instead
    // of registers through the K loop, where register pressure would spill
    // them to scratch, whose reloads wait for every load in flight (the
    // next tile's chunks)
    __shared__ __align__(1024) uint8_t lds[kSqBufs * kSqBuf + kThreads * 16];
    v4u* const lconst = reinterpret_cast<v4u*>(lds + kSqBufs * kSqBuf);
    uint32_t* sOut = reinterpret_cast<uint32_t*>(lds + 2 * kSqBuf);  // buffers 2 and 3

    const int g = blockIdx.z;
    const uint8_t* A = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.A) + g * a.strideA);
    const uint8_t* B = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.B) + g * a.strideB);
    uint32_t* C = static_cast<uint32_t*>(a.C) + g * a.strideC;
    const uint32_t p = a.p[g];
    const double inv_p = ex.inv_p[g];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (w & 1) * 64, wc = (w >> 1) * 32;
    const uint64_t rowBytes = uint64_t(4) << a.s;
    const int nk_all = 1 << (a.s - 6);  // chunks of 64 entries
    const int nk = nk_all / splits;
    const int kc0 = int(blockIdx.y) * nk;
    const uint64_t tilesA = uint64_t(1) << (a.fA - 7), tilesB = uint64_t(1) << (a.fB - 7);
    const uint64_t T = tilesA * tilesB;
    if (uint64_t(blockIdx.x) >= T) return;

    // output mapping: tile-local t = 4 tid + k + 2048 q (k < 4, q < 8) at
    // position pdep(t, TM), TM = the 7 lowest A bits and 7 lowest B bits of
    // C; the 7 lowest bits of C are always tile bits, so k adds to the
    // position and each thread writes four consecutive words per q
    const uint64_t TM = pdep64(127, a.maskA) | pdep64(127, a.maskB);
    const uint64_t offLow = pdep64(uint64_t(4 * tid), TM);
    const uint32_t iLow = uint32_t(pext64(offLow, a.maskA)), jLow = uint32_t(pext64(offLow, a.maskB));
    // loads: lane l of wave w fills physical slot l % 8 of row 8 w + l / 8,
    // i.e. logical slot c = (l % 8) ^ ((l / 8) % 8): bytes 16 c.. of the
    // row's chunk (plane c / 4)
    const uint32_t ldRow = uint32_t(8 * w + (lane >> 3));
    const uint32_t ldSlot = uint32_t((lane & 7) ^ ((lane >> 3) & 7));
    const uint32_t voff = ldRow * uint32_t(rowBytes) + 16 * ldSlot;
    const uint64_t rows64 = 64 * rowBytes;
    uint8_t* const ldsW = lds + w * 1024;
    const int fr = lane & 15, q = lane >> 4;
    const int sw[kDigits] = {((0 + q) ^ (fr & 7)) * 16, ((4 + q) ^ (fr & 7)) * 16};
    // output staging: the residue of tile-local (i, j) sits at word
    // stage_pos(i, j), a linear (XOR) map chosen on the host so that both the
    // MFMA-layout writes and the C-order reads of a wave hit 64 distinct banks
    auto stage_pos = [&](uint32_t i, uint32_t j) {
        uint32_t x = 0;
#pragma unroll
        for (int b = 0; b < 7; ++b) {
            x ^= ((i >> b) & 1u) ? ex.phiI[b] : 0u;
            x ^= ((j >> b) & 1u) ? ex.phiJ[b] : 0u;
        }
        return x;
    };
    lconst[tid] = v4u{stage_pos(uint32_t(wr + 4 * q), uint32_t(wc + fr)), stage_pos(iLow, jLow),
                      uint32_t(offLow), uint32_t(offLow >> 32)};
    __syncthreads();

    uint64_t tile = blockIdx.x, ta, tb;
    tile_coords(tile, tilesA, tilesB, ta, tb);
    const uint8_t* tA = A + ta * kSqM * rowBytes;
    const uint8_t* tB = B + tb * kSqN * rowBytes;
    sq_fetch(tA, tB, uint64_t(kc0), rows64, voff, ldsW);
    if (nk > 1) sq_fetch(tA, tB, uint64_t(kc0 + 1), rows64, voff, ldsW + kSqBuf);

    for (;;) {
        v4i acc[kShifts][4][2];
#pragma unroll
        for (int t = 0; t < kShifts; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[t][i][j] = v4i{0, 0, 0, 0};

        // chunk 0 has landed (chunk 1 may be in flight), and every wave is
        // done with the previous tile's output staging in buffers 2 and 3
        if (nk > 1)
            chunk_barrier<kSqLoads>();
        else
            chunk_barrier<0>();
        if (nk > 2) sq_fetch(tA, tB, uint64_t(kc0 + 2), rows64, voff, ldsW + 2 * kSqBuf);
        if (nk > 3) sq_fetch(tA, tB, uint64_t(kc0 + 3), rows64, voff, ldsW + 3 * kSqBuf);
        SqFrags f0, f1;
        sq_read(lds, wr, wc, fr, sw, f0);

        const uint64_t next = tile + gridDim.x;
        const bool more = next < T;
        uint64_t nta = 0, ntb = 0;
        const uint8_t *nA = tA, *nB = tB;

        // chunk kc (fragments in cur) while chunk kc + 1 is read into nxt
        auto step = [&](int kc, SqFrags& cur, SqFrags& nxt) {
            // chunk kc + 1 has landed (up to two later ones may be in
            // flight) and no wave reads chunk kc any more: its buffer takes
            // chunk kc + 4
            const int ahead = nk - 2 - kc;
            if (ahead >= 2)
                chunk_barrier<2 * kSqLoads>();
            else if (ahead == 1)
                chunk_barrier<kSqLoads>();
            else
                chunk_barrier<0>();
            if (kc + 4 < nk) sq_fetch(tA, tB, uint64_t(kc0 + kc + 4), rows64, voff, ldsW + (kc & 3) * kSqBuf);
            sq_read(lds + ((kc + 1) & 3) * kSqBuf, wr, wc, fr, sw, nxt);
            sq_mfma(cur, acc);
            if (((kc + 1) & (kSqFlush - 1)) == 0) flush(acc, p, inv_p);
        };
        // the tile's last chunk: every fragment is in registers, so buffers
        // 0 and 1 take the next tile's first chunks
        auto last = [&](SqFrags& cur) {
            chunk_barrier<63>();
            if (more) {
                tile_coords(next, tilesA, tilesB, nta, ntb);
                nA = A + nta * kSqM * rowBytes;
                nB = B + ntb * kSqN * rowBytes;
                sq_fetch(nA, nB, uint64_t(kc0), rows64, voff, ldsW);
                if (nk > 1) sq_fetch(nA, nB, uint64_t(kc0 + 1), rows64, voff, ldsW + kSqBuf);
            }
            sq_mfma(cur, acc);
        };
        int kc = 0;
        for (; kc + 2 < nk; kc += 2) {
            step(kc, f0, f1);
            step(kc + 1, f1, f0);
        }
        if (kc + 1 < nk) {
            step(kc, f0, f1);
            last(f1);
        } else {
            last(f0);
        }

        // epilogue: lane holds rows 4 (lane / 16) + v, column lane % 16 of
        // each 16x16 block; the residues are staged, then written in C order
        // (split K: partial residues in C order within the tile)
        {
            // per tile, like the store addresses below
            int ci = tid;
            __asm__ volatile("" : "+v"(ci));  // read here, per tile
            const v4u lc = lconst[ci];
            const uint32_t wP = lc.x;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        int32_t Tt[kShifts];
#pragma unroll
                        for (int t = 0; t < kShifts; ++t) Tt[t] = acc[t][rb][cb][v];
                        // i = wr + 4 q + (16 rb + v), j = wc + fr + 16 cb
                        const uint32_t u = ((v & 1) ? ex.phiI[0] : 0u) ^ ((v & 2) ? ex.phiI[1] : 0u) ^
                                           ((rb & 1) ? ex.phiI[4] : 0u) ^ ((rb & 2) ? ex.phiI[5] : 0u) ^
                                           (cb ? ex.phiJ[4] : 0u);
                        sOut[wP ^ u] = combine_digits(Tt, p, inv_p);
                        // one residue at a time: scheduled together, the 96
                        // conversions to double would need twice the
                        // accumulators' registers
                        __builtin_amdgcn_sched_barrier(0);
                    }
            // staging complete (the next tile's loads may stay in flight)
            chunk_barrier<63>();
            const uint64_t baseC = pdep64(ta * kSqM, a.maskA) | pdep64(tb * kSqN, a.maskB);
            uint4* pt = reinterpret_cast<uint4*>(part + blockIdx.z * part_stride +
                                                 (uint64_t(blockIdx.y) * T + tile) * (kSqM * kSqN));
            // the store addresses are formed here, per tile: hoisted out of
            // the tile loop they would hold 48 registers through the K loop
            const uint64_t oLow = uint64_t(lc.z) | (uint64_t(lc.w) << 32);
            const uint32_t rP = lc.y;
#pragma unroll
            for (int qq = 0; qq < 8; ++qq) {
                const uint64_t o = oLow | ex.hiOff[qq];
                const uint32_t r = rP ^ ex.stageQ[qq];
                const uint32_t v[4] = {sOut[r], sOut[r ^ ex.stageK[1]], sOut[r ^ ex.stageK[2]],
                                       sOut[r ^ ex.stageK[3]]};
                if (splits > 1) {
                    pt[tid + 512 * qq] = uint4{v[0], v[1], v[2], v[3]};
                    continue;
                }
                const uint64_t e = baseC | o;
                if (ex.digits_out) {
                    uint32_t wd[kDigits];
                    digit_words(v, p, wd);
                    uint32_t* cw = C + (e >> 6) * 64 + ((e & 63) >> 2);
#pragma unroll
                    for (int d = 0; d < kDigits; ++d) cw[16 * d] = wd[d];
                } else {
                    *reinterpret_cast<uint4*>(C + e) = uint4{v[0], v[1], v[2], v[3]};
                }
            }
        }
        if (!more) break;
        tile = next;
        ta = nta;
        tb = ntb;
        tA = nA;
        tB = nB;
    }
}

// split-K: add the partial residues of every K range and scatter into C
// (tiles of 128 x BN; partial tiles in (i, j) order for BN = 64, in C order
// within the tile for BN = 128)
template <int BN>
__global__ __launch_bounds__(256) void k_mfma_reduce(StepArgs a, const uint32_t* part, int64_t part_stride,
                                                     int splits, int digits_out) {
    const int g = blockIdx.z;
    const uint32_t p = a.p[g];
    uint32_t* C = static_cast<uint32_t*>(a.C) + g * a.strideC;
    const uint64_t tilesA = uint64_t(1) << (a.fA - 7), tilesB = uint64_t(1) << (a.fB - (BN == 128 ? 7 : 6));
    const uint64_t T = tilesA * tilesB;
    const uint64_t n = T * (kBM * BN);
    const uint32_t* pg = part + g * part_stride;
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t tile = e / (kBM * BN), loc = e % (kBM * BN);
        uint64_t sum = 0;
        for (int y = 0; y < splits; ++y) sum += pg[(uint64_t(y) * T + tile) * (kBM * BN) + loc];
        uint64_t ta, tb;
        tile_coords(tile, tilesA, tilesB, ta, tb);
        uint64_t c;
        if (BN == 128) {
            const uint64_t TM = pdep64(127, a.maskA) | pdep64(127, a.maskB);
            c = pdep64(ta * kBM, a.maskA) | pdep64(tb * BN, a.maskB) | pdep64(loc, TM);
        } else {
            const uint64_t i = loc / BN, j = loc % BN;
            c = pdep64(ta * kBM + i, a.maskA) | pdep64(tb * BN + j, a.maskB);
        }
        const uint32_t r = uint32_t(sum % p);
        if (digits_out) {
            // entry c's digit d at byte 256 (c / 64) + 64 d + c % 64
            const int32_t x = r > (p >> 1) ? int32_t(r - p) : int32_t(r);
            const int32_t d0 = int32_t(int8_t(x & 0xff));
            uint8_t* cb = reinterpret_cast<uint8_t*>(C) + (c >> 6) * 256 + (c & 63);
            cb[0] = uint8_t(uint32_t(d0) & 0xffu);
            cb[64] = uint8_t(uint32_t((x - d0) >> 8) & 0xffu);
        } else {
            C[c] = r;
        }
    }
}

namespace {

// rank over GF(2) of a set of 6-bit values
int rank6(const uint32_t* v, int n) {
    uint32_t basis[6] = {0, 0, 0, 0, 0, 0};
    int r = 0;
    for (int a = 0; a < n; ++a) {
        uint32_t x = v[a] & 63u;
        for (int b = 5; b >= 0 && x; --b) {
            if (!((x >> b) & 1u)) continue;
            if (!basis[b]) {
                basis[b] = x;
                ++r;
                break;
            }
            x ^= basis[b];
        }
    }
    return r;
}

// Staging layout of a 128 x 128 output tile. Word of tile-local (i, j):
// bits 7.. = i, bit 6 = j6, bank bits 0..5 = j0..j5 XOR M (i0..i6, j6),
// a bijection for any 6 x 8 bit matrix M. A wave's staging writes vary in
// (i2, i3, j0..j3) (lane / 16 and lane % 16 of the MFMA layout) and its
// C-order reads in the tile bits at C-order positions 2..7 (consecutive
// lanes read consecutive groups of four words); M is drawn (from a fixed
// seed) until both sets map onto all 6 bank bits, so neither access has a
// bank conflict. Without such an M the layout stays correct (M = 0).
void stage_layout(const StepArgs& a, uint64_t TM, MfmaExtra& ex) {
    // tile bit at C-order position t: i (A side) or j (B side) and its index
    int isA[14], idx[14];
    int p = 0, ni = 0, nj = 0;
    for (int b = 0; b < 64 && p < 14; ++b) {
        if (!((TM >> b) & 1u)) continue;
        isA[p] = int((a.maskA >> b) & 1u);
        idx[p] = isA[p] ? ni++ : nj++;
        ++p;
    }
    uint32_t M[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // columns: i0..i6, j6
    auto image = [&](int A_side, int k) -> uint32_t {
        if (A_side) return M[k];
        return k < 6 ? (1u << k) : M[7];
    };
    uint32_t rng = 0x2545f491u;
    for (int attempt = 0; attempt < 20000; ++attempt) {
        for (int c = 0; c < 8; ++c) {
            rng ^= rng << 13;
            rng ^= rng >> 17;
            rng ^= rng << 5;
            M[c] = rng & 63u;
        }
        const uint32_t W[6] = {image(1, 2), image(1, 3), image(0, 0), image(0, 1), image(0, 2), image(0, 3)};
        uint32_t R[6];
        for (int t = 2; t < 8; ++t) R[t - 2] = image(isA[t], idx[t]);
        if (rank6(W, 6) == 6 && rank6(R, 6) == 6) break;
        if (attempt == 19999)
            for (int c = 0; c < 8; ++c) M[c] = 0;
    }
    for (int k = 0; k < 7; ++k) {
        ex.phiI[k] = (1u << (7 + k)) | M[k];
        ex.phiJ[k] = k < 6 ? (1u << k) : ((1u << 6) | M[7]);
    }
    auto pos = [&](uint32_t i, uint32_t j) {
        uint32_t x = 0;
        for (int b = 0; b < 7; ++b) {
            if ((i >> b) & 1u) x ^= ex.phiI[b];
            if ((j >> b) & 1u) x ^= ex.phiJ[b];
        }
        return x;
    };
    for (int q = 0; q < 8; ++q) ex.stageQ[q] = pos(ex.hiI[q], ex.hiJ[q]);
    for (int k = 0; k < 4; ++k) ex.stageK[k] = pos(ex.dI[k], ex.dJ[k]);
}

}  // namespace

hipError_t launch_mfma(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                       double step_macs, char* scratch, int64_t scratch_per_plane, unsigned dig) {
    MfmaExtra ex{};
    ex.digits_out = (dig & 4u) ? 1u : 0u;
    for (int g = 0; g < G; ++g) {
        ex.inv_p[g] = 1.0 / double(a.p[g]);
    }
    auto pdep = [](uint64_t x, uint64_t m) {
        uint64_t r = 0;
        for (; m; m &= m - 1, x >>= 1)
            if (x & 1) r |= m & (~m + 1);
        return r;
    };
    auto pext = [](uint64_t x, uint64_t m) {
        uint64_t r = 0, bit = 1;
        for (; m; m &= m - 1, bit <<= 1)
            if (x & m & (~m + 1)) r |= bit;
        return r;
    };
    // 128 x 128 tiles when both free sides allow them (and a tile's rows
    // span less than 4 GiB: the square kernel's load offsets are 32-bit)
    const bool sq = a.fB >= 7 && a.s <= 24;
    const int bn = sq ? kSqN : kBN;
    const uint64_t TM = pdep(127, a.maskA) | pdep(uint64_t(bn - 1), a.maskB);
    for (int q = 0; q < (sq ? 8 : 4); ++q) {
        ex.hiOff[q] = pdep(uint64_t(q) << 11, TM);
        ex.hiI[q] = uint32_t(pext(ex.hiOff[q], a.maskA));
        ex.hiJ[q] = uint32_t(pext(ex.hiOff[q], a.maskB));
    }
    for (int q = 0; q < 4; ++q) {
        ex.dI[q] = uint32_t(pext(uint64_t(q), a.maskA));
        ex.dJ[q] = uint32_t(pext(uint64_t(q), a.maskB));
    }
    if (sq) stage_layout(a, TM, ex);
    const uint64_t T = (uint64_t(1) << (a.fA - 7)) * (uint64_t(1) << (a.fB - (sq ? 7 : 6)));
    // too few output tiles to fill the GPU: split K over block rows (powers
    // of two, as many partial tiles per plane as the scratch area holds, at
    // least one stage each)
    int splits = 1;
    const int nk = sq ? 1 << (a.s - 6) : a.s >= 7 ? 1 << (a.s - 7) : 1;
    const uint64_t cap_tiles = uint64_t(scratch_per_plane) / (4 * kBM * uint64_t(bn));
    // the 128 x 64 kernel sums at most 2^15 entries (256 stages) per block row
    if (!sq)
        while (nk / splits > (1 << 15) / 128) splits *= 2;
    if (T * uint64_t(splits) > cap_tiles && splits > 1) return hipErrorInvalidValue;
    while (T * G * splits * 2 <= 1024 && splits * 2 <= nk && T * splits * 2 <= cap_tiles) splits *= 2;
    const uint64_t nA = (uint64_t(1) << (a.fA + a.s)) / 4, nB = (uint64_t(1) << (a.fB + a.s)) / 4;
    auto blocks = [](uint64_t n) { return dim3(uint32_t(std::min<uint64_t>((n + 255) / 256, 1u << 16)), 1, 1); };
    dim3 gA = blocks(nA), gB = blocks(nB);
    gA.z = gB.z = G;
    // the digit pass reads and rewrites in place the operands that are not
    // digit planes already (those came from a matrix-core step's epilogue)
    hipError_t e = hipSuccess;
    if ((dig & 3u) != 3u) {
        prof->before(stream);
        if (!(dig & 1u)) {
            hipLaunchKernelGGL(k_digits, gA, dim3(256), 0, stream, static_cast<uint32_t*>(const_cast<void*>(a.A)),
                               a.strideA, nA, a);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (!(dig & 2u)) {
            hipLaunchKernelGGL(k_digits, gB, dim3(256), 0, stream, static_cast<uint32_t*>(const_cast<void*>(a.B)),
                               a.strideB, nB, a);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const double n4 = double((dig & 1u) ? 0 : nA) + double((dig & 2u) ? 0 : nB);
        prof->after_raw(stream, KC_DIGITS, 2.0 * 16.0 * n4 * G, 0.0);
    }
    uint32_t* part = reinterpret_cast<uint32_t*>(scratch);
    const int64_t part_stride = scratch_per_plane / 4;
    dim3 grid(uint32_t(std::min<uint64_t>(T, 1024)), uint32_t(splits), G);
    prof->before(stream);
    if (sq)
        hipLaunchKernelGGL(k_mfma_sq, grid, dim3(kThreads), 0, stream, a, ex, splits, part, part_stride);
    else if (a.s >= 7)
        hipLaunchKernelGGL(k_mfma<true>, grid, dim3(kThreads), 0, stream, a, ex, splits, part, part_stride);
    else
        hipLaunchKernelGGL(k_mfma<false>, grid, dim3(kThreads), 0, stream, a, ex, splits, part, part_stride);
    if (splits > 1) {
        const uint64_t n = T * (kBM * uint64_t(bn));
        dim3 gr(uint32_t(std::min<uint64_t>((n + 255) / 256, 4096)), 1, G);
        if (sq)
            hipLaunchKernelGGL(k_mfma_reduce<kSqN>, gr, dim3(256), 0, stream, a, part, part_stride, splits,
                               int(ex.digits_out));
        else
            hipLaunchKernelGGL(k_mfma_reduce<kBN>, gr, dim3(256), 0, stream, a, part, part_stride, splits,
                               int(ex.digits_out));
    }
    prof->after_raw(stream, KC_MFMA, step_bytes, step_macs);
    return hipGetLastError();
}

bool mfma_eligible(const StepArgs& a, int el) { return el == EL_I8 ? mfma8_eligible(a) : mfma_eligible(a); }

bool mfma_eligible(const StepArgs& a) {
    // 128 x 128 tiles: K up to 2^24 (32-bit load offsets within a tile).
    // 128 x 64 tiles (B's free side of 6 bits): K split into ranges of 2^15
    // whose partial tiles (2^(fA - 7) per range, 32 KiB each) fit the 4 MiB
    // scratch of a prime
    return a.s >= 6 && a.fA >= 7 &&
           ((a.fB >= 7 && a.s <= 24) || (a.fB == 6 && (a.s <= 15 || (a.fA - 7) + (a.s - 15) <= 7)));
}

}  // namespace tn
