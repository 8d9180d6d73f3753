// Narrow dense steps on the matrix cores, for residues modulo small moduli
// (m <= 255, centred int8 values): C[xA, j] = sum_z A[z | xA] B[z | j] with
// few B rows (2^fB <= 64) and a shared dimension of at least 64 entries
// (Sec. 2.1, Eq. 5 form; all shared bonds at once). Per residue plane the
// step is a tall matrix times a narrow one: A, 2^fA rows of K bytes, is the
// only large operand, and every one of its bytes meets at most 64 B rows.
// Such a step is bound by reading A, so the kernel reads A exactly once,
// straight from global memory into the registers of the wave that uses it, in
// whole 128-byte lines (a lane takes 32 consecutive bytes of a row, four lanes
// a line, sixteen rows per wave instruction); B is re-read from the L2 by
// every work-group. One v_mfma_i32_16x16x64_i8 per 16 x 16 block takes a lane's
// 16 bytes of A and of B at the same K offsets, so the products it sums are
// those of a contraction over 64 entries whatever K offsets each lane holds;
// two per 128-byte chunk. Sums of up to 2^16 products (each at most 127^2)
// stay exact in int32 (< 2^30); longer K is reduced to centred residues every
// 2^16 entries. Steps with too few row tiles to fill the GPU split K over
// block rows (partial residues in scratch, then a reduction kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.hpp"
#include "mfma.hpp"
#include "profile.hpp"

namespace tn {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kRowBlocks = 4;                            // 16-row blocks per wave
constexpr int kWaves = 4;                                // waves per work-group
constexpr int kTileRows = 16 * kRowBlocks * kWaves;      // A rows per work-group tile
constexpr int kExactBytes = 1 << 16;                     // K entries summed exactly in int32

// a lane's share of one row in one chunk: KB = 32 (two MFMAs, 128-byte
// chunks) or 16 (one MFMA, 64-byte chunks when K = 64)
template <int KB>
struct Frag {
    v4i x[KB / 16];
};

template <int KB>
__device__ __forceinline__ Frag<KB> load_frag(const int8_t* p) {
    Frag<KB> f;
#pragma unroll
    for (int i = 0; i < KB / 16; ++i) f.x[i] = *reinterpret_cast<const v4i*>(p + 16 * i);
    return f;
}

// CB: 16-row blocks of B (2^fB rows rounded up to 16; rows beyond 2^fB read
// B's last row and are never stored). Tiles of kTileRows A rows are dealt to
// the work-groups; blockIdx.y is the K range (of `splits`), blockIdx.z the
// residue plane.
template <int CB, int KB>
__global__ __launch_bounds__(256) void k_mfma8_narrow(StepArgs a, int splits, int8_t* part, int64_t part_stride) {
    constexpr int RA = kRowBlocks;
    constexpr int CHUNK = 4 * KB;  // bytes of a row per chunk
    __shared__ uint64_t dA[kTileRows];
    __shared__ uint64_t dB[16 * CB];
    const int g = blockIdx.z;
    const int8_t* A = static_cast<const int8_t*>(a.A) + g * a.strideA;
    const int8_t* B = static_cast<const int8_t*>(a.B) + g * a.strideB;
    int8_t* C = static_cast<int8_t*>(a.C) + g * a.strideC;
    const ModSmall ms{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fr = lane & 15, q = lane >> 4;
    const uint64_t K = uint64_t(1) << a.s;
    const uint64_t rowsA = uint64_t(1) << a.fA;
    const int nB = 1 << a.fB;
    const uint64_t T = (rowsA + kTileRows - 1) / kTileRows;
    // output bit deposits of tile-local A indices and of B indices
    for (int i = tid; i < kTileRows; i += 256) dA[i] = pdep64(uint64_t(i), a.maskA);
    for (int i = tid; i < 16 * CB; i += 256) dB[i] = pdep64(uint64_t(i), a.maskB);
    __syncthreads();
    const uint64_t nchunks = K / CHUNK;
    const uint64_t per = nchunks / uint64_t(splits);
    const uint64_t c0 = per * blockIdx.y;
    const uint64_t kofs = c0 * CHUNK + uint64_t(q) * KB;
    const int8_t* pb[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) pb[cb] = B + uint64_t(std::min(16 * cb + fr, nB - 1)) * K + kofs;
    const uint64_t flush = kExactBytes / CHUNK;

    for (uint64_t tile = blockIdx.x; tile < T; tile += gridDim.x) {
        const uint64_t row0 = tile * kTileRows + uint64_t(w) * 16 * RA;
        const int8_t* pa[RA];
#pragma unroll
        for (int rb = 0; rb < RA; ++rb)
            pa[rb] = A + std::min<uint64_t>(row0 + 16 * rb + fr, rowsA - 1) * K + kofs;
        v4i acc[RA][CB];
#pragma unroll
        for (int rb = 0; rb < RA; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = v4i{0, 0, 0, 0};
        Frag<KB> xa[2][RA], xb[2][CB];
        auto load = [&](int buf, uint64_t c) {
            const uint64_t o = c * CHUNK;
#pragma unroll
            for (int rb = 0; rb < RA; ++rb) xa[buf][rb] = load_frag<KB>(pa[rb] + o);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) xb[buf][cb] = load_frag<KB>(pb[cb] + o);
        };
        auto mma = [&](int buf) {
#pragma unroll
            for (int i = 0; i < KB / 16; ++i)
#pragma unroll
                for (int rb = 0; rb < RA; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[rb][cb] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(xa[buf][rb].x[i], xb[buf][cb].x[i], acc[rb][cb], 0, 0, 0);
        };
        auto reduce_all = [&]() {
#pragma unroll
            for (int rb = 0; rb < RA; ++rb)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[rb][cb][v] = ms.center32(acc[rb][cb][v]);
        };
        // chunks in pairs, the next chunk's loads issued before the current
        // chunk's products; every `flush` chunks the sums become residues
        load(0, 0);
        uint64_t c = 0;
        while (c < per) {
            if (c + 1 < per) load(1, c + 1);
            mma(0);
            if (++c % flush == 0 && c < per) reduce_all();
            if (c >= per) break;
            if (c + 1 < per) load(0, c + 1);
            mma(1);
            if (++c % flush == 0 && c < per) reduce_all();
        }
        // epilogue: lane holds A rows row0 + 16 rb + 4 q + v, B row 16 cb + fr
        const uint64_t tA = pdep64(tile * kTileRows, a.maskA);
        const int la = w * 16 * RA + 4 * q;
#pragma unroll
        for (int rb = 0; rb < RA; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t xa_ = tile * kTileRows + uint64_t(la + 16 * rb + v);
                if (xa_ >= rowsA) continue;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int j = 16 * cb + fr;
                    if (j >= nB) continue;
                    const int8_t r = int8_t(ms.center32(acc[rb][cb][v]));
                    if (splits > 1)
                        part[g * part_stride + int64_t(blockIdx.y) * int64_t(rowsA) * nB + int64_t(xa_) * nB + j] = r;
                    else
                        C[tA | dA[la + 16 * rb + v] | dB[j]] = r;
                }
            }
    }
}

// split K: add the partial residues of every range and store into C
__global__ __launch_bounds__(256) void k_narrow8_reduce(StepArgs a, const int8_t* part, int64_t part_stride,
                                                        int splits) {
    const int g = blockIdx.z;
    int8_t* C = static_cast<int8_t*>(a.C) + g * a.strideC;
    const ModSmall ms{int32_t(a.p[g]), a.r2[g], a.r16[g], a.pinv[g]};
    const uint64_t n = uint64_t(1) << (a.fA + a.fB);
    const int8_t* p = part + g * part_stride;
    for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += uint64_t(gridDim.x) * blockDim.x) {
        int32_t sum = 0;  // at most 64 partial residues of magnitude <= 127
        for (int k = 0; k < splits; ++k) sum += p[uint64_t(k) * n + e];
        const uint64_t xa = e >> a.fB, j = e & ((uint64_t(1) << a.fB) - 1);
        C[pdep64(xa, a.maskA) | pdep64(j, a.maskB)] = int8_t(ms.center32(sum));
    }
}

template <int CB, int KB>
hipError_t launch_cb(const StepArgs& a, int G, hipStream_t stream, char* scratch, int64_t scratch_per_plane) {
    const uint64_t rowsA = uint64_t(1) << a.fA;
    const uint64_t T = (rowsA + kTileRows - 1) / kTileRows;
    const uint64_t nchunks = (uint64_t(1) << a.s) / (4 * KB);
    const uint64_t outs = rowsA << a.fB;
    // split K until the launch has about 1024 work-groups, each range keeping
    // at least 8 chunks and the partial residues fitting the scratch area
    int splits = 1;
    while (T * uint64_t(G) * splits < 1024 && nchunks / (uint64_t(splits) * 2) >= 8 &&
           outs * uint64_t(splits) * 2 <= uint64_t(scratch_per_plane) && splits < 64)
        splits *= 2;
    dim3 grid(uint32_t(std::min<uint64_t>(T, 2048)), uint32_t(splits), uint32_t(G));
    int8_t* part = reinterpret_cast<int8_t*>(scratch);
    hipLaunchKernelGGL((k_mfma8_narrow<CB, KB>), grid, dim3(256), 0, stream, a, splits, part, scratch_per_plane);
    if (splits > 1) {
        dim3 gr(uint32_t(std::min<uint64_t>((outs + 255) / 256, 4096)), 1, uint32_t(G));
        hipLaunchKernelGGL(k_narrow8_reduce, gr, dim3(256), 0, stream, a, part, scratch_per_plane, splits);
    }
    return hipGetLastError();
}

template <int KB>
hipError_t launch_kb(const StepArgs& a, int G, hipStream_t stream, char* scratch, int64_t scratch_per_plane) {
    if (a.fB <= 4) return launch_cb<1, KB>(a, G, stream, scratch, scratch_per_plane);
    if (a.fB == 5) return launch_cb<2, KB>(a, G, stream, scratch, scratch_per_plane);
    return launch_cb<4, KB>(a, G, stream, scratch, scratch_per_plane);
}

}  // namespace

bool narrow8_eligible(const StepArgs& a) {
    // B side of at most 64 rows (steps with a wider B and at least 128 A rows
    // go to the tiled kernel), K of at least 64 entries, A rows within 32-bit
    // tile counts
    return a.s >= 6 && a.s <= 40 && a.fA >= a.fB && a.fA <= 40 && (a.fB <= 5 || (a.fB == 6 && a.fA < 7));
}

hipError_t launch_narrow8(const StepArgs& a, int G, hipStream_t stream, Profiler* prof, double step_bytes,
                          double step_macs, char* scratch, int64_t scratch_per_plane) {
    if (!narrow8_eligible(a)) return hipErrorInvalidValue;
    prof->before(stream);
    const hipError_t e = a.s == 6 ? launch_kb<16>(a, G, stream, scratch, scratch_per_plane)
                                  : launch_kb<32>(a, G, stream, scratch, scratch_per_plane);
    prof->after_raw(stream, KC_NARROW, step_bytes, step_macs);
    return e;
}

}  // namespace tn
