// Residue number system: prime table and Chinese remaindering into a big
// integer (little-endian base-2^32 limbs).
//
// Every entry of every intermediate tensor is a count of partial
// assignments, at most 2^n for n variables, so the final count is at most
// 2^n and residues modulo primes whose product exceeds 2^n determine it.
// The primes are the largest ones below kPrimeBound = 65280: their centred
// residues (|r| <= 32639) are exactly two signed base-256 digits, which is
// what the matrix-core kernel multiplies, and being above 2^16 - 2^11 they
// allow the kernels' folding reduction (2^16 = 2^16 - p mod p, below 2^11).
// primes_needed(n) is the fewest leading primes whose product exceeds 2^n.
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace tn {

static bool is_prime_u32(uint32_t q) {
    if (q < 2) return false;
    if (q % 2 == 0) return q == 2;
    for (uint32_t f = 3; uint64_t(f) * f <= q; f += 2)
        if (q % f == 0) return false;
    return true;
}

const std::vector<uint32_t>& prime_table(int32_t k) {
    static std::mutex mu;
    static std::vector<uint32_t> table;
    std::lock_guard<std::mutex> lk(mu);
    uint32_t q = table.empty() ? kPrimeBound - 1 : table.back() - 1;
    while (int32_t(table.size()) < k) {
        if (is_prime_u32(q)) table.push_back(q);
        --q;
    }
    return table;
}

int32_t primes_needed(int32_t n_vars) {
    const std::vector<uint32_t>& P = prime_table(TN_MAX_PRIMES);
    double bits = 0.0;
    int32_t k = 0;
    // a margin of one bit over n absorbs any rounding in the logarithms
    while (k < TN_MAX_PRIMES && bits <= double(n_vars) + 1.0) bits += std::log2(double(P[size_t(k++)]));
    return bits > double(n_vars) + 1.0 ? k : TN_MAX_PRIMES + 1;
}

static uint32_t powmod(uint64_t b, uint64_t e, uint32_t p) {
    uint64_t r = 1;
    b %= p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return uint32_t(r);
}

void crt_limbs(const uint32_t* residues, int32_t k, std::vector<uint32_t>& limbs) {
    const std::vector<uint32_t>& P = prime_table(k);
    // Garner: x = v0 + v1 p0 + v2 p0 p1 + ... with 0 <= vi < pi
    std::vector<uint32_t> v(k);
    for (int32_t i = 0; i < k; ++i) {
        uint64_t pi = P[i];
        uint64_t x = residues[i] % pi;
        for (int32_t j = 0; j < i; ++j) {
            uint64_t inv = powmod(P[j] % pi, pi - 2, uint32_t(pi));
            x = (x + pi - v[j] % pi) % pi * inv % pi;
        }
        v[i] = uint32_t(x);
    }
    limbs.assign(1, 0);
    for (int32_t i = k - 1; i >= 0; --i) {
        // limbs = limbs * p_i + v_i  (Horner over the mixed radix)
        uint64_t carry = v[i];
        uint64_t mul = (i == k - 1) ? 0 : P[i];
        if (i == k - 1) {
            limbs[0] = v[i];
            continue;
        }
        for (auto& l : limbs) {
            uint64_t t = uint64_t(l) * mul + carry;
            l = uint32_t(t);
            carry = t >> 32;
        }
        if (carry) limbs.push_back(uint32_t(carry));
    }
    while (limbs.size() > 1 && limbs.back() == 0) limbs.pop_back();
}

}  // namespace tn
