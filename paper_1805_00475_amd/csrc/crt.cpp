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
//
// Counts up to about 2^333 use small moduli instead: pairwise coprime
// integers of at most 255 (255, 254, 253, 251, 247, ..., taken greedily
// from the top), whose centred residues (|r| <= 127) are single int8
// values. A modular multiply-add is then one int8 product rather than four
// digit products, at the price of about twice as many residue planes.
// Chinese remaindering needs the moduli pairwise coprime only, not prime.
#include <cmath>
#include <numeric>
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

const std::vector<uint32_t>& small_moduli() {
    static const std::vector<uint32_t> table = [] {
        std::vector<uint32_t> t;
        for (uint32_t m = kSmallModulusMax; m >= 2; --m) {
            bool coprime = true;
            for (uint32_t c : t) coprime = coprime && std::gcd(m, c) == 1u;
            if (coprime) t.push_back(m);
        }
        return t;
    }();
    return table;
}

int32_t small_moduli_needed(int32_t n_vars) {
    const std::vector<uint32_t>& M = small_moduli();
    double bits = 0.0;
    int32_t k = 0;
    while (k < int32_t(M.size()) && bits <= double(n_vars) + 1.0) bits += std::log2(double(M[size_t(k++)]));
    return bits > double(n_vars) + 1.0 ? k : 0;
}

// inverse of a modulo m (gcd(a, m) = 1), by the extended Euclidean algorithm
static uint64_t inverse_mod(uint64_t a, uint64_t m) {
    int64_t r0 = int64_t(m), r1 = int64_t(a % m), t0 = 0, t1 = 1;
    while (r1 != 0) {
        const int64_t q = r0 / r1;
        const int64_t r2 = r0 - q * r1, t2 = t0 - q * t1;
        r0 = r1;
        r1 = r2;
        t0 = t1;
        t1 = t2;
    }
    return uint64_t(t0 < 0 ? t0 + int64_t(m) : t0);
}

void crt_limbs(const uint32_t* residues, int32_t k, std::vector<uint32_t>& limbs) {
    crt_limbs(residues, prime_table(k).data(), k, limbs);
}

void crt_limbs(const uint32_t* residues, const uint32_t* P, int32_t k, std::vector<uint32_t>& limbs) {
    // Garner: x = v0 + v1 m0 + v2 m0 m1 + ... with 0 <= vi < mi
    std::vector<uint32_t> v(k);
    for (int32_t i = 0; i < k; ++i) {
        uint64_t pi = P[i];
        uint64_t x = residues[i] % pi;
        for (int32_t j = 0; j < i; ++j) {
            uint64_t inv = inverse_mod(P[j] % pi, pi);
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
