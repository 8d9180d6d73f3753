// Device arithmetic and kernel argument blocks for the contraction step
// C[xA, xB] = sum_z A[z | xA] * B[z | xB] (Sec. 2.1, Eq. 5 form), with every
// tensor stored in the plan's death-order layout (shared bonds = low s bits).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

constexpr int kMaxGroup = 16;  // primes per launch (gridDim.z)

struct StepArgs {
    const void* A;
    const void* B;
    void* C;
    int64_t strideA, strideB, strideC;  // elements between prime planes (0 = shared)
    uint64_t maskA, maskB;              // C bits taken from A / from B
    int32_t rC, s, fA, fB;              // output rank, shared bonds, free bits of A and B
    uint32_t p[kMaxGroup];              // primes of this launch (RNS)
    uint32_t r2[kMaxGroup];             // 2^32 mod p (small for p close to 2^31)
};

// Residues modulo p = 2^31 - d with 2d < 2^12. A 64-bit value x = h 2^32 + l
// is congruent to h (2^32 mod p) + l, which is below 2^45 (fold). Three
// products below 2^62 added to a folded value stay below 2^64, so the
// accumulator folds after every third product. Two folds bring any 64-bit
// value below 2^32 + 2^25 < 3p; two conditional subtractions finish.
struct ModP {
    uint32_t p, r;
    __device__ __forceinline__ uint64_t fold(uint64_t x) const { return (x >> 32) * r + (x & 0xffffffffull); }
    __device__ __forceinline__ uint32_t finish(uint64_t x) const {
        x = fold(fold(x));
        const uint64_t p2 = uint64_t(p) << 1;
        x = x >= p2 ? x - p2 : x;
        x = x >= p ? x - p : x;
        return uint32_t(x);
    }
};

// Scatter the low bits of x into the set bits of mask (bit deposit).
__device__ __forceinline__ uint64_t pdep64(uint64_t x, uint64_t mask) {
    uint64_t r = 0;
    while (mask) {
        uint64_t low = mask & (~mask + 1);
        if (x & 1) r |= low;
        x >>= 1;
        mask &= mask - 1;
    }
    return r;
}

// Gather the bits of x at the set bits of mask into the low bits (extract).
__device__ __forceinline__ uint64_t pext64(uint64_t x, uint64_t mask) {
    uint64_t r = 0, bit = 1;
    while (mask) {
        uint64_t low = mask & (~mask + 1);
        if (x & low) r |= bit;
        bit <<= 1;
        mask &= mask - 1;
    }
    return r;
}

}  // namespace tn
