// Dense contraction steps on the matrix cores, exactly.
//
// A step whose shared dimension K = 2^s is wide and whose two free sides are
// large is a plain matrix product C = A B^T over residues modulo p < 2^31
// (rows of A and B are contiguous along the shared bonds in the plan's
// layout). Each residue r is centred to r' in (-p/2, p/2] and written as four
// signed base-256 digits r' = d0 + d1 2^8 + d2 2^16 + d3 2^24 with d0..d2 in
// [-128, 127] and |d3| <= 64. Then
//     C = sum over t = 0..6 of 2^(8t) T_t,   T_t = sum_{i+j=t} A_i B_j^T,
// where A_i, B_j are int8 digit matrices; every T_t is accumulated by the
// int8 MFMA into int32 registers. Each product of digits is at most 2^14 in
// magnitude, at most four digit pairs share a shift, so K <= 2^14 keeps every
// T_t below 2^30 -- exact; wider K is summed in chunks of 2^14 whose results
// are reduced to residues and added modulo p. The epilogue forms
//     X = (T0 + T1 2^8 + T2 2^16 + T3 2^24) + (T4 + T5 2^8 + T6 2^16) (2^32 mod p)
// in 64-bit integers (|X| < 2^59), adds a multiple of p above 2^59, and
// reduces with the folding reduction of the other kernels.
//
// Two kernels per step: k_digits rewrites A and B in place (they die at this
// step) so that every 64-entry chunk of a row holds its four digit planes of
// 64 bytes each; k_mfma then copies digit tiles into LDS and runs
// v_mfma_i32_16x16x64_i8. Output tiles are staged in LDS and written in
// C-address order so stores stay coalesced for any bit interleaving.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "mfma.hpp"
#include "profile.hpp"

namespace tn {

typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------- digit pass
// In place: the 16 lanes owning one 64-entry chunk read it (4 entries each)
// before any of them writes, since they are consecutive lanes of one wave
// and every store depends on all four loads of that lane.
__global__ __launch_bounds__(256) void k_digits(uint32_t* X, int64_t stride, uint64_t n_vec4,
                                                StepArgs a) {
    const uint32_t p = a.p[blockIdx.z];
    uint32_t* base = X + blockIdx.z * stride;
    const uint32_t half = p >> 1;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < n_vec4;
         v += uint64_t(gridDim.x) * blockDim.x) {
        uint4 r = reinterpret_cast<const uint4*>(base)[v];
        uint32_t rv[4] = {r.x, r.y, r.z, r.w};
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int32_t c = rv[e] > half ? int32_t(rv[e] - p) : int32_t(rv[e]);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                int32_t dig = d < 3 ? int32_t(int8_t(c & 0xff)) : c;
                w[d] |= (uint32_t(dig) & 0xffu) << (8 * e);
                c = (c - dig) >> 8;
            }
        }
        // chunk = 16 vec4 of 64 entries; plane d of the chunk at byte 64 d
        const uint64_t chunk = v >> 4;
        const uint32_t lane16 = uint32_t(v & 15);
        uint32_t* cbase = base + chunk * 64;
#pragma unroll
        for (int d = 0; d < 4; ++d) cbase[d * 16 + lane16] = w[d];
    }
}

// --------------------------------------------------------------- GEMM
// Work-group tile 128 (xA) x 64 (xB), 8 waves of 32 x 32 (two per SIMD), K
// consumed in chunks of 64 entries (one 16x16x64 MFMA per digit pair and
// 16x16 block). Digit tiles are double-buffered in LDS: the global loads of
// chunk k+1 are issued before the MFMAs of chunk k and stored to the other
// buffer after them, one barrier per chunk.
constexpr int kBM = 128, kBN = 64, kRowB = 256 + 16;  // LDS row stride (bytes)
constexpr int kBuf = (kBM + kBN) * kRowB;             // one LDS buffer
constexpr int kThreads = 512;

// V = sum_t 2^(8t) T_t is congruent to sum_t T_t w_t with w_t = 2^(8t) mod p:
// w_0..w_3 = 1, 2^8, 2^16, 2^24 and w_4..w_6 = r, r 2^8, r 2^16 with
// r = 2^32 mod p < 2^12. Every |T_t| < 2^30 (|T_6| < 2^26), so every term is
// below 2^55 in magnitude and seven signed 32x32->64 multiply-adds are
// exact; adding off (a multiple of p of at least 2^59) makes the sum
// positive for the folding reduction.
__device__ __forceinline__ uint32_t combine_digits(const int32_t T[7], uint32_t p, uint32_t r, uint64_t off) {
    const int32_t ri = int32_t(r);
    int64_t x = int64_t(T[0]);
    x += int64_t(T[1]) * 256;
    x += int64_t(T[2]) * 65536;
    x += int64_t(T[3]) * 16777216;
    x += int64_t(T[4]) * int64_t(ri);
    x += int64_t(T[5]) * int64_t(ri << 8);
    x += int64_t(T[6]) * int64_t(ri << 16);
    const ModP m{p, r};
    return m.finish(uint64_t(x) + off);
}

constexpr int kFlushChunks = (1 << 14) / 64;  // K chunks of 64 per exact int32 accumulation

// Tile traversal. Work-groups are dealt to the 8 XCDs round-robin, so tile
// t runs on XCD t % 8. Each XCD owns a band of A tiles (or of B tiles when
// there are fewer than 8 A tiles) and walks it in groups of up to 8 tiles of
// that side: the group stays in the XCD's L2 while the other operand's tiles
// stream past it once per group.
__device__ __forceinline__ void tile_coords(uint64_t tile, uint64_t tilesA, uint64_t tilesB, uint64_t& ta,
                                            uint64_t& tb) {
    if (tilesA < 8 && tilesB < 8) {
        ta = tile % tilesA;
        tb = tile / tilesA;
        return;
    }
    const uint64_t x = tile & 7, j = tile >> 3;
    if (tilesA >= 8) {
        const uint64_t per = tilesA >> 3;
        const uint64_t gm = per < 8 ? per : 8;
        const uint64_t span = gm * tilesB;
        const uint64_t group = j / span, r = j % span;
        ta = x * per + group * gm + r % gm;
        tb = r / gm;
    } else {
        const uint64_t per = tilesB >> 3;
        const uint64_t gn = per < 8 ? per : 8;
        const uint64_t span = gn * tilesA;
        const uint64_t group = j / span, r = j % span;
        tb = x * per + group * gn + r % gn;
        ta = r / gn;
    }
}

__device__ __forceinline__ void flush(v4i (&acc)[7][2][2], uint32_t (&racc)[2][2][4], uint32_t p, uint32_t r2,
                                      uint64_t off) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int32_t Tt[7];
#pragma unroll
                for (int t = 0; t < 7; ++t) Tt[t] = acc[t][rb][cb][v];
                const uint32_t x = combine_digits(Tt, p, r2, off) + racc[rb][cb][v];
                racc[rb][cb][v] = x >= p ? x - p : x;
            }
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) acc[t][rb][cb] = v4i{0, 0, 0, 0};
}

__global__ __launch_bounds__(kThreads, 1) void k_mfma(StepArgs a, MfmaExtra ex, int splits, uint32_t* part,
                                                      int64_t part_stride) {
    __shared__ __align__(16) uint8_t lds[2 * kBuf];
    __shared__ uint64_t hiOff[16];
    __shared__ uint32_t hiIJ[16][2];
    uint32_t* sOut = reinterpret_cast<uint32_t*>(lds);  // kBM x kBN after the K loop

    const int g = blockIdx.z;
    const uint8_t* A = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.A) + g * a.strideA);
    const uint8_t* B = reinterpret_cast<const uint8_t*>(static_cast<const uint32_t*>(a.B) + g * a.strideB);
    uint32_t* C = static_cast<uint32_t*>(a.C) + g * a.strideC;
    const uint32_t p = a.p[g], r2 = a.r2[g];
    const uint64_t off = ex.off[g];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 3) * 32, wc = (w >> 2) * 32;
    const uint64_t rowBytes = uint64_t(4) << a.s;  // K entries of 4 bytes (4 digit planes)
    const int nk_all = 1 << (a.s - 6);
    // split-K: block row blockIdx.y owns chunks [kc0, kc0 + nk)
    const int nk = nk_all / splits;
    const int kc0 = int(blockIdx.y) * nk;
    const uint64_t tilesA = uint64_t(1) << (a.fA - 7), tilesB = uint64_t(1) << (a.fB - 6);
    const uint64_t T = tilesA * tilesB;

    // output mapping inside a tile: tile-local t = tid | q << 9 (q < 16),
    // position pdep(t, TM), TM = the 7 lowest A bits and 6 lowest B bits of C
    const uint64_t TM = pdep64(127, a.maskA) | pdep64(63, a.maskB);
    const uint64_t offLow = pdep64(uint64_t(tid), TM);
    const uint32_t iLow = uint32_t(pext64(offLow, a.maskA)), jLow = uint32_t(pext64(offLow, a.maskB));
    if (tid < 16) {
        const uint64_t oh = pdep64(uint64_t(tid) << 9, TM);
        hiOff[tid] = oh;
        hiIJ[tid][0] = uint32_t(pext64(oh, a.maskA));
        hiIJ[tid][1] = uint32_t(pext64(oh, a.maskB));
    }
    // raw digit copies: thread tid moves 16 B at row (tid / 16) + 32 q,
    // byte (tid % 16) * 16 of the 256-byte chunk (A: q < 4, B: q < 2)
    const int ldRow = tid >> 4, ldCol = (tid & 15) * 16;
    const int kg = (lane >> 4) * 16;
    const int fr = lane & 15;
    __syncthreads();

    for (uint64_t tile = blockIdx.x; tile < T; tile += gridDim.x) {
        uint64_t ta, tb;
        tile_coords(tile, tilesA, tilesB, ta, tb);
        const uint64_t xA0 = ta * kBM, xB0 = tb * kBN;
        const uint8_t* gA = A + xA0 * rowBytes;
        const uint8_t* gB = B + xB0 * rowBytes;

        v4i acc[7][2][2];
        uint32_t racc[2][2][4];  // residues of the K chunks already flushed
#pragma unroll
        for (int t = 0; t < 7; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[t][i][j] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) racc[i][j][v] = 0;

        // prefetch registers (named, so they stay in VGPRs)
        uint4 pa0, pa1, pa2, pa3, pb0, pb1;
#define TN_FETCH(kc_)                                                                         \
    do {                                                                                      \
        const uint64_t kb_ = uint64_t(kc_) * 256 + ldCol;                                     \
        pa0 = *reinterpret_cast<const uint4*>(gA + uint64_t(ldRow) * rowBytes + kb_);         \
        pa1 = *reinterpret_cast<const uint4*>(gA + uint64_t(ldRow + 32) * rowBytes + kb_);    \
        pa2 = *reinterpret_cast<const uint4*>(gA + uint64_t(ldRow + 64) * rowBytes + kb_);    \
        pa3 = *reinterpret_cast<const uint4*>(gA + uint64_t(ldRow + 96) * rowBytes + kb_);    \
        pb0 = *reinterpret_cast<const uint4*>(gB + uint64_t(ldRow) * rowBytes + kb_);         \
        pb1 = *reinterpret_cast<const uint4*>(gB + uint64_t(ldRow + 32) * rowBytes + kb_);    \
    } while (0)
#define TN_STASH(buf_)                                                                        \
    do {                                                                                      \
        uint8_t* sA_ = lds + (buf_) * kBuf;                                                   \
        uint8_t* sB_ = sA_ + kBM * kRowB;                                                     \
        *reinterpret_cast<uint4*>(sA_ + ldRow * kRowB + ldCol) = pa0;                         \
        *reinterpret_cast<uint4*>(sA_ + (ldRow + 32) * kRowB + ldCol) = pa1;                  \
        *reinterpret_cast<uint4*>(sA_ + (ldRow + 64) * kRowB + ldCol) = pa2;                  \
        *reinterpret_cast<uint4*>(sA_ + (ldRow + 96) * kRowB + ldCol) = pa3;                  \
        *reinterpret_cast<uint4*>(sB_ + ldRow * kRowB + ldCol) = pb0;                         \
        *reinterpret_cast<uint4*>(sB_ + (ldRow + 32) * kRowB + ldCol) = pb1;                  \
    } while (0)
        __syncthreads();  // the previous tile's output staging is done with the LDS
        TN_FETCH(kc0);
        TN_STASH(0);
        __syncthreads();
        for (int kc = 0; kc < nk; ++kc) {
            const int buf = kc & 1;
            if (kc + 1 < nk) TN_FETCH(kc0 + kc + 1);
            const uint8_t* sA = lds + buf * kBuf;
            const uint8_t* sB = sA + kBM * kRowB;
            v4i fa[4][2], fb[4][2];
#pragma unroll
            for (int d = 0; d < 4; ++d)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    fa[d][b] = *reinterpret_cast<const v4i*>(sA + (wr + b * 16 + fr) * kRowB + d * 64 + kg);
                    fb[d][b] = *reinterpret_cast<const v4i*>(sB + (wc + b * 16 + fr) * kRowB + d * 64 + kg);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[i + j][rb][cb] =
                                __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i][rb], fb[j][cb], acc[i + j][rb][cb], 0, 0, 0);
            // every 2^14 entries of K, fold the exact int32 sums into residues
            // so they never exceed 2^30
            if (((kc + 1) & (kFlushChunks - 1)) == 0 && kc + 1 < nk) flush(acc, racc, p, r2, off);
            if (kc + 1 < nk) TN_STASH(buf ^ 1);
            __syncthreads();
        }
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
                        int32_t Tt[7];
#pragma unroll
                        for (int t = 0; t < 7; ++t) Tt[t] = acc[t][rb][cb][v];
                        const int i = wr + rb * 16 + 4 * (lane >> 4) + v;
                        const int j = wc + cb * 16 + fr;
                        const uint32_t x = combine_digits(Tt, p, r2, off) + racc[rb][cb][v];
                        pt[i * kBN + j] = x >= p ? x - p : x;
                    }
            continue;
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int32_t Tt[7];
#pragma unroll
                    for (int t = 0; t < 7; ++t) Tt[t] = acc[t][rb][cb][v];
                    const int i = wr + rb * 16 + 4 * (lane >> 4) + v;
                    const int j = wc + cb * 16 + fr;
                    const uint32_t x = combine_digits(Tt, p, r2, off) + racc[rb][cb][v];  // < 2p < 2^32
                    sOut[i * kBN + j] = x >= p ? x - p : x;
                }
        __syncthreads();
        const uint64_t baseC = pdep64(xA0, a.maskA) | pdep64(xB0, a.maskB);
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
            const uint64_t o = offLow | hiOff[q];
            const uint32_t i = iLow | hiIJ[q][0];
            const uint32_t j = jLow | hiIJ[q][1];
            C[baseC | o] = sOut[i * kBN + j];
        }
    }
#undef TN_FETCH
#undef TN_STASH
}

// split-K: add the partial residues of every K range and scatter into C
__global__ __launch_bounds__(256) void k_mfma_reduce(StepArgs a, const uint32_t* part, int64_t part_stride,
                                                     int splits) {
    const int g = blockIdx.z;
    const uint32_t p = a.p[g];
    uint32_t* C = static_cast<uint32_t*>(a.C) + g * a.strideC;
    const uint64_t tilesA = uint64_t(1) << (a.fA - 7), tilesB = uint64_t(1) << (a.fB - 6);
    const uint64_t T = tilesA * tilesB;
    const uint64_t n = T * (kBM * kBN);
    const uint32_t* pg = part + g * part_stride;
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t tile = e / (kBM * kBN), loc = e % (kBM * kBN);
        uint64_t sum = 0;
        for (int y = 0; y < splits; ++y) sum += pg[(uint64_t(y) * T + tile) * (kBM * kBN) + loc];
        uint64_t ta, tb;
        tile_coords(tile, tilesA, tilesB, ta, tb);
        const uint64_t i = loc / kBN, j = loc % kBN;
        C[pdep64(ta * kBM + i, a.maskA) | pdep64(tb * kBN + j, a.maskB)] = uint32_t(sum % p);
    }
}

hipError_t launch_mfma(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                       double step_macs, char* scratch, int64_t scratch_per_plane) {
    MfmaExtra ex{};
    for (int g = 0; g < G; ++g) {
        const uint64_t p = a.p[g];
        ex.off[g] = p * ((uint64_t(1) << 59) / p + 1);
    }
    const uint64_t nA = (uint64_t(1) << (a.fA + a.s)) / 4, nB = (uint64_t(1) << (a.fB + a.s)) / 4;
    auto blocks = [](uint64_t n) { return dim3(uint32_t(std::min<uint64_t>((n + 255) / 256, 1u << 16)), 1, 1); };
    dim3 gA = blocks(nA), gB = blocks(nB);
    gA.z = gB.z = G;
    prof->before(stream);
    hipLaunchKernelGGL(k_digits, gA, dim3(256), 0, stream, static_cast<uint32_t*>(const_cast<void*>(a.A)),
                       a.strideA, nA, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_digits, gB, dim3(256), 0, stream, static_cast<uint32_t*>(const_cast<void*>(a.B)),
                       a.strideB, nB, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the digit pass reads and rewrites both operands in place
    prof->after_raw(stream, KC_DIGITS, 2.0 * 16.0 * double(nA + nB) * G, 0.0);
    const uint64_t T = (uint64_t(1) << (a.fA - 7)) * (uint64_t(1) << (a.fB - 6));
    // too few output tiles to fill the GPU: split K over block rows (powers
    // of two, at most 128 partial tiles per plane in the scratch area, at
    // least one 64-entry chunk each)
    int splits = 1;
    const int nk = 1 << (a.s - 6);
    const uint64_t cap_tiles = uint64_t(scratch_per_plane) / (4 * kBM * kBN);
    while (T * G * splits * 2 <= 1024 && splits * 2 <= nk && T * splits * 2 <= cap_tiles) splits *= 2;
    uint32_t* part = reinterpret_cast<uint32_t*>(scratch);
    const int64_t part_stride = scratch_per_plane / 4;
    dim3 grid(uint32_t(std::min<uint64_t>(T, 1024)), uint32_t(splits), G);
    prof->before(stream);
    hipLaunchKernelGGL(k_mfma, grid, dim3(kThreads), 0, stream, a, ex, splits, part, part_stride);
    if (splits > 1) {
        const uint64_t n = T * (kBM * kBN);
        dim3 gr(uint32_t(std::min<uint64_t>((n + 255) / 256, 4096)), 1, G);
        hipLaunchKernelGGL(k_mfma_reduce, gr, dim3(256), 0, stream, a, part, part_stride, splits);
    }
    prof->after_raw(stream, KC_MFMA, step_bytes, step_macs);
    return hipGetLastError();
}

bool mfma_eligible(const StepArgs& a) {
    return a.s >= 6 && a.fA >= 7 && a.fB >= 6;
}

}  // namespace tn
