// Device helpers shared by the matrix-core kernels (mfma.hip, mfma8.hip):
// tile traversal, LDS barriers with explicit wait counts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

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

// The same traversal for tile counts 2^lgA and 2^lgB, in shifts and masks.
__device__ __forceinline__ void tile_coords_lg(uint32_t tile, int lgA, int lgB, uint32_t& ta, uint32_t& tb) {
    if (lgA < 3 && lgB < 3) {
        ta = tile & ((1u << lgA) - 1);
        tb = tile >> lgA;
        return;
    }
    const uint32_t x = tile & 7, j = tile >> 3;
    const int lper = (lgA >= 3 ? lgA : lgB) - 3;    // log2 of the band per XCD
    const int lg = lper < 3 ? lper : 3;              // log2 of the group size
    const int lspan = lg + (lgA >= 3 ? lgB : lgA);  // log2 of tiles per group
    const uint32_t group = j >> lspan, r = j & ((1u << lspan) - 1);
    const uint32_t own = (x << lper) + (group << lg) + (r & ((1u << lg) - 1)), other = r >> lg;
    ta = lgA >= 3 ? own : other;
    tb = lgA >= 3 ? other : own;
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// s_waitcnt immediate: vector memory count <= vm (0..63), LDS count 0
constexpr int wait_vm_lgkm0(int vm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4); }

// Chunk barrier: the waiting wave's loads into LDS, except the newest VM of
// them, have landed and its LDS reads have returned; then all waves meet.
// After it, every wave's data of the awaited chunk is in LDS and no wave
// still reads a buffer that is about to be refilled. The empty asm
// statements keep the compiler from moving memory accesses across it; the
// fence of __syncthreads is not used because it would also wait for the
// loads still in flight.
template <int VM>
__device__ __forceinline__ void chunk_barrier() {
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(VM));
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

}  // namespace tn
