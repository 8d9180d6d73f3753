// Device arithmetic and kernel argument blocks for the contraction step
// C[xA, xB] = sum_z A[z | xA] * B[z | xB] (Sec. 2.1, Eq. 5 form), with every
// tensor stored in the plan's death-order layout (shared bonds = low s bits).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

constexpr int kMaxGroup = 16;  // residue planes per launch (gridDim.z)

// Element kinds of a contraction: residues modulo 16-bit primes (u32),
// 64-bit wrapping counts, or centred residues modulo small moduli (int8).
enum ElemKind : int { EL_U32 = 0, EL_U64 = 1, EL_I8 = 2 };
template <int E>
struct ElemT;
template <>
struct ElemT<EL_U32> {
    using T = uint32_t;
};
template <>
struct ElemT<EL_U64> {
    using T = uint64_t;
};
template <>
struct ElemT<EL_I8> {
    using T = int8_t;
};

struct StepArgs {
    const void* A;
    const void* B;
    void* C;
    int64_t strideA, strideB, strideC;  // elements between residue planes (0 = shared)
    uint64_t maskA, maskB;              // C bits taken from A / from B
    int32_t rC, s, fA, fB;              // output rank, shared bonds, free bits of A and B
    uint32_t p[kMaxGroup];              // moduli of this launch (RNS)
    uint32_t r2[kMaxGroup];             // 2^32 mod p
    uint32_t r16[kMaxGroup];            // 2^16 mod p (small moduli)
    float pinv[kMaxGroup];              // 1 / p (small moduli)
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

// Centred residue of a signed sum modulo a small modulus m <= 255, in
// (-m/2, m/2] (so |r| <= 127, an int8). x = h 2^16 + l with 0 <= l < 2^16 is
// congruent to h r16 + l (r16 = 2^16 mod m < 256); from |x| < 2^31 one fold
// gives |y| < 2^24, exact in single precision, where y / m floors to a
// quotient off by at most one (the product's relative error is below
// 2^-23 and |y / m| < 2^17), so y - q m lies in [-m, 2m): one conditional
// add or subtract gives [0, m), one more the centred range. Wider sums
// first fold at 2^32 (r32 = 2^32 mod m) down to 31 bits.
struct ModSmall {
    int32_t m;
    uint32_t r32, r16;
    float inv;
    __device__ __forceinline__ int32_t center32(int32_t x) const {
        const int32_t y = (x >> 16) * int32_t(r16) + (x & 0xffff);
        const int32_t q = int32_t(floorf(float(y) * inv));
        int32_t r = y - q * m;
        r += r < 0 ? m : 0;
        r -= r >= m ? m : 0;
        r -= r > (m >> 1) ? m : 0;
        return r;
    }
    __device__ __forceinline__ int32_t center64(int64_t x) const {
        // |x| < 2^63: two folds at 2^32 bring it below 2^40.1, then 2^31
        x = (x >> 32) * int64_t(r32) + int64_t(x & 0xffffffffll);
        x = (x >> 32) * int64_t(r32) + int64_t(x & 0xffffffffll);
        const int32_t y = int32_t((x >> 16) * int64_t(r16)) + int32_t(x & 0xffff);
        return center32(y);
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
