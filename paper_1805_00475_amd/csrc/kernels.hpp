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

// Residues modulo primes p in (2^16 - 2^11, 2^16), r = 2^32 mod p < 2^16.
// A 64-bit value x = h 2^32 + l is congruent to h r + l, below 2^48 + 2^32
// (fold); products of residues are below 2^32, so a folded accumulator
// takes at least 2^15 more products before it could overflow (the kernels
// fold after every third). To finish, a second fold brings x below 2^33,
// and four folds at 2^16 (2^16 = 2^16 - p mod p, below 2^11) bring it
// below 2^33 -> 2^28.01 -> 2^23.02 -> 2^18.35 -> 75776 < 2p; one
// conditional subtraction ends below p.
struct ModP {
    uint32_t p, r;
    __device__ __forceinline__ uint64_t fold(uint64_t x) const { return (x >> 32) * r + (x & 0xffffffffull); }
    __device__ __forceinline__ uint32_t finish(uint64_t x) const {
        x = fold(fold(x));
        const uint32_t r16 = 65536u - p;
        uint32_t y = uint32_t(x >> 16) * r16 + uint32_t(x & 0xffffu);  // < 2^28.01
        y = (y >> 16) * r16 + (y & 0xffffu);
        y = (y >> 16) * r16 + (y & 0xffffu);
        y = (y >> 16) * r16 + (y & 0xffffu);
        return y >= p ? y - p : y;
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
