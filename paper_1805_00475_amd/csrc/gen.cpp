// Seeded synthetic instances (Sec. 3.2 workloads): uniform random cubic
// graphs, vertex cover of a cubic graph as 2-variable OR clauses, monotone
// 1-in-3 with uniform clauses, and the paper's own 1-in-3 family (one
// variable per edge of a cubic graph, one exactly-one clause per vertex).
//
// Random numbers: SplitMix64 expands a 64-bit seed into the state of
// xoshiro256** (Blackman and Vigna); a bounded draw rejects the biased low
// range of the 64-bit output. Cubic graphs come from the configuration model
// (3n stubs shuffled by Fisher-Yates, consecutive stubs paired) with the
// whole draw rejected on a self-loop or a repeated edge, which samples
// simple cubic graphs uniformly. These steps are the published definitions
// of the generators; the Python package ``instances`` implements the same
// definitions, and a test checks that both emit identical formulas.
#include <cstdint>
#include <set>
#include <utility>
#include <vector>

#include "tn.h"

namespace {

uint64_t splitmix_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Xoshiro {
    uint64_t s[4];
    explicit Xoshiro(uint64_t seed) {
        uint64_t st = seed;
        for (auto& w : s) w = splitmix_next(st);
    }
    uint64_t next() {
        const uint64_t result = rotl(s[1] * 5, 7) * 9;
        const uint64_t t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return result;
    }
    // uniform in [0, n): reject draws at or above the largest multiple of n
    uint64_t below(uint64_t n) {
        const uint64_t rem = (~uint64_t(0) - n + 1) % n;  // 2^64 mod n
        const uint64_t limit = rem ? uint64_t(0) - rem : 0;  // 0 stands for 2^64
        for (;;) {
            const uint64_t x = next();
            if (limit == 0 || x < limit) return x % n;
        }
    }
};

// configuration model with rejection; edges as (min, max) in pairing order
bool cubic_edges(int32_t n, uint64_t seed, std::vector<std::pair<int32_t, int32_t>>& edges) {
    Xoshiro rng(seed);
    std::vector<int32_t> stubs(size_t(3) * size_t(n));
    for (int tries = 0; tries < 100000; ++tries) {
        for (int32_t v = 0; v < n; ++v)
            for (int k = 0; k < 3; ++k) stubs[size_t(3 * v + k)] = v;
        for (size_t i = stubs.size() - 1; i > 0; --i) {
            const size_t j = size_t(rng.below(uint64_t(i) + 1));
            std::swap(stubs[i], stubs[j]);
        }
        edges.clear();
        std::set<std::pair<int32_t, int32_t>> seen;
        bool ok = true;
        for (size_t i = 0; i < stubs.size(); i += 2) {
            const int32_t u = stubs[i], v = stubs[i + 1];
            if (u == v) {
                ok = false;
                break;
            }
            const std::pair<int32_t, int32_t> e(std::min(u, v), std::max(u, v));
            if (!seen.insert(e).second) {
                ok = false;
                break;
            }
            edges.push_back(e);
        }
        if (ok) return true;
    }
    return false;
}

}  // namespace

extern "C" {

uint64_t tn_instance_seed(int32_t family, uint64_t index, uint64_t master) {
    uint64_t st = master ^ (uint64_t(uint32_t(family)) << 40) ^ index;
    return splitmix_next(st);
}

tn_status tn_gen_cubic_graph(int32_t n, uint64_t seed, int32_t* edges) {
    if (n < 4 || n % 2 || n > (1 << 24) || !edges) return TN_EINVAL;
    std::vector<std::pair<int32_t, int32_t>> e;
    try {
        if (!cubic_edges(n, seed, e)) return TN_EUNSUPPORTED;
    } catch (...) {
        return TN_ENOMEM;
    }
    for (size_t i = 0; i < e.size(); ++i) {
        edges[2 * i] = e[i].first;
        edges[2 * i + 1] = e[i].second;
    }
    return TN_OK;
}

tn_status tn_gen_exactly_one_3(int32_t n, int32_t m, uint64_t seed, int32_t* clause_ptr, int32_t* lits,
                               uint8_t* kinds) {
    if (n < 0 || m < 0 || (m > 0 && n < 3) || m > (1 << 28) || !clause_ptr || (m > 0 && (!lits || !kinds)))
        return TN_EINVAL;
    Xoshiro rng(seed);
    clause_ptr[0] = 0;
    for (int32_t c = 0; c < m; ++c) {
        const int32_t a = int32_t(rng.below(uint64_t(n)));
        int32_t b = int32_t(rng.below(uint64_t(n)));
        while (b == a) b = int32_t(rng.below(uint64_t(n)));
        int32_t d = int32_t(rng.below(uint64_t(n)));
        while (d == a || d == b) d = int32_t(rng.below(uint64_t(n)));
        lits[3 * c] = a + 1;
        lits[3 * c + 1] = b + 1;
        lits[3 * c + 2] = d + 1;
        kinds[c] = TN_CLAUSE_EXACTLY_ONE;
        clause_ptr[c + 1] = 3 * (c + 1);
    }
    return TN_OK;
}

tn_status tn_gen_cubic_vc(int32_t n, uint64_t seed, int32_t* clause_ptr, int32_t* lits, uint8_t* kinds) {
    if (!clause_ptr || !lits || !kinds) return TN_EINVAL;
    std::vector<int32_t> e(size_t(3) * size_t(std::max(n, 0)));
    const tn_status st = tn_gen_cubic_graph(n, seed, e.data());
    if (st != TN_OK) return st;
    const int32_t m = 3 * n / 2;
    clause_ptr[0] = 0;
    for (int32_t c = 0; c < m; ++c) {
        lits[2 * c] = e[size_t(2 * c)] + 1;
        lits[2 * c + 1] = e[size_t(2 * c + 1)] + 1;
        kinds[c] = TN_CLAUSE_OR;
        clause_ptr[c + 1] = 2 * (c + 1);
    }
    return TN_OK;
}

tn_status tn_gen_cubic_1in3(int32_t n_vertices, uint64_t seed, int32_t* clause_ptr, int32_t* lits,
                            uint8_t* kinds) {
    if (!clause_ptr || !lits || !kinds) return TN_EINVAL;
    const int32_t n = n_vertices;
    std::vector<int32_t> e(size_t(3) * size_t(std::max(n, 0)));
    const tn_status st = tn_gen_cubic_graph(n, seed, e.data());
    if (st != TN_OK) return st;
    // variable i + 1 is edge i; each vertex's clause lists its incident
    // edges in increasing edge order
    std::vector<int32_t> fill(size_t(n), 0);
    for (int32_t i = 0; i < 3 * n / 2; ++i)
        for (int k = 0; k < 2; ++k) {
            const int32_t v = e[size_t(2 * i + k)];
            lits[3 * v + fill[size_t(v)]++] = i + 1;
        }
    clause_ptr[0] = 0;
    for (int32_t v = 0; v < n; ++v) {
        kinds[v] = TN_CLAUSE_EXACTLY_ONE;
        clause_ptr[v + 1] = 3 * (v + 1);
    }
    return TN_OK;
}

}  // extern "C"
