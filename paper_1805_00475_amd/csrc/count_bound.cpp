// Upper bound on the count of a boolean formula, used to size the residue
// system: the count is recovered from its residues modulo moduli whose
// product exceeds the bound (Sec. 2.1, the count as the full trace; Sec. 3.2
// on exactness), so a tighter bound means fewer residue planes.
//
// The variables are split into blocks of at most kBlock. For an assignment x
// every clause value is 0 or 1, and a satisfied clause passes these tests on
// the restriction of x to any block B: a clause lying inside B is satisfied
// there, and an exactly-one clause that only partly lies in B has at most one
// true literal there. Hence the product of the clause values is at most the
// product over blocks of the indicator that x|B passes every test of B, and
// summing over x, the count is at most the product over blocks of the number
// of assignments of B passing its tests. Clauses that use a variable twice
// are left out of the tests (a relaxation), and an empty clause makes the
// count 0. Each block is counted by bit slicing: 64 assignments of its six
// lowest variables per machine word.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace tn {

namespace {

constexpr int kBlock = 16;

struct Test {
    int kind;        // TN_CLAUSE_*
    bool inside;     // every literal in the block
    uint32_t pos;    // block variables of positive literals
    uint32_t neg;    // block variables of negative literals
};

// lane patterns of the six lowest block variables over 64 assignments
constexpr uint64_t kLane[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                               0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

uint64_t count_block(int k, const std::vector<Test>& tests) {
    const int low = std::min(k, 6);
    const uint64_t lanes = low == 6 ? ~uint64_t(0) : ((uint64_t(1) << (1 << low)) - 1);
    uint64_t word[kBlock];
    uint64_t total = 0;
    for (uint64_t h = 0; h < (uint64_t(1) << (k - low)); ++h) {
        for (int j = 0; j < k; ++j) word[j] = j < 6 ? kLane[j] : (((h >> (j - 6)) & 1) ? ~uint64_t(0) : 0);
        uint64_t ok = lanes;
        for (const Test& t : tests) {
            uint64_t one = 0, two = 0, any = 0;  // odd count, two or more, at least one
            for (int j = 0; j < k; ++j) {
                uint64_t lit;
                if ((t.pos >> j) & 1) lit = word[j];
                else if ((t.neg >> j) & 1) lit = ~word[j];
                else continue;
                two |= one & lit;
                one ^= lit;
                any |= lit;
            }
            if (t.kind == TN_CLAUSE_OR) ok &= any;
            else if (t.kind == TN_CLAUSE_EXACTLY_ONE) ok &= t.inside ? (one & ~two) : ~two;
            else ok &= one;  // parity
            if (!ok) break;
        }
        total += uint64_t(__builtin_popcountll(ok));
    }
    return total;
}

}  // namespace

int32_t count_bound_bits(const tn_formula* f) {
    const int32_t n = f->n_vars, m = f->n_clauses;
    std::vector<std::vector<int32_t>> cl_of(static_cast<size_t>(n));
    std::vector<char> usable(static_cast<size_t>(m), 1);
    for (int32_t c = 0; c < m; ++c) {
        const int32_t b = f->clause_ptr[c], e = f->clause_ptr[c + 1];
        if (b == e) return 0;  // an empty clause: the count is 0
        for (int32_t i = b; i < e; ++i)
            for (int32_t j = b; j < i; ++j)
                if (std::abs(f->lits[i]) == std::abs(f->lits[j])) usable[size_t(c)] = 0;
        if (!usable[size_t(c)]) continue;
        for (int32_t i = b; i < e; ++i) cl_of[size_t(std::abs(f->lits[i]) - 1)].push_back(c);
    }
    // blocks grown greedily from the unplaced variable in most clauses,
    // adding the neighbour that completes most clauses (touching ones count
    // half); ties to the lowest index
    std::vector<int32_t> block_of(static_cast<size_t>(n), -1);
    std::vector<std::vector<int32_t>> blocks;
    std::vector<int32_t> order(static_cast<size_t>(n));
    for (int32_t v = 0; v < n; ++v) order[size_t(v)] = v;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return cl_of[size_t(a)].size() > cl_of[size_t(b)].size(); });
    for (int32_t s : order) {
        if (block_of[size_t(s)] >= 0) continue;
        const int32_t id = int32_t(blocks.size());
        blocks.push_back({s});
        block_of[size_t(s)] = id;
        std::vector<int32_t>& blk = blocks.back();
        while (int(blk.size()) < kBlock) {
            int32_t best = -1;
            double bs = -1;
            for (size_t bi = 0; bi < blk.size(); ++bi)
                for (int32_t c : cl_of[size_t(blk[bi])])
                    for (int32_t i = f->clause_ptr[c]; i < f->clause_ptr[c + 1]; ++i) {
                        const int32_t u = std::abs(f->lits[i]) - 1;
                        if (block_of[size_t(u)] >= 0) continue;
                        double sc = 0;
                        for (int32_t c2 : cl_of[size_t(u)]) {
                            bool all = true, touch = false;
                            for (int32_t j = f->clause_ptr[c2]; j < f->clause_ptr[c2 + 1]; ++j) {
                                const int32_t w = std::abs(f->lits[j]) - 1;
                                const bool in = w == u || block_of[size_t(w)] == id;
                                all = all && in;
                                touch = touch || (w != u && in);
                            }
                            sc += all ? 1.0 : touch ? 0.5 : 0.0;
                        }
                        if (sc > bs || (sc == bs && u < best)) {
                            bs = sc;
                            best = u;
                        }
                    }
            if (best < 0) break;
            block_of[size_t(best)] = id;
            blk.push_back(best);
        }
    }
    double bits = 0;
    std::vector<int32_t> pos_in(static_cast<size_t>(n), -1);
    for (const auto& blk : blocks) {
        const int k = int(blk.size());
        for (int j = 0; j < k; ++j) pos_in[size_t(blk[size_t(j)])] = j;
        std::vector<int32_t> seen;
        std::vector<Test> tests;
        for (int32_t v : blk)
            for (int32_t c : cl_of[size_t(v)]) {
                if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
                seen.push_back(c);
                Test t{f->kinds[c], true, 0, 0};
                int inside = 0;
                for (int32_t i = f->clause_ptr[c]; i < f->clause_ptr[c + 1]; ++i) {
                    const int32_t l = f->lits[i], w = std::abs(l) - 1;
                    const int32_t p = block_of[size_t(w)] == block_of[size_t(v)] ? pos_in[size_t(w)] : -1;
                    if (p < 0) {
                        t.inside = false;
                        continue;
                    }
                    ++inside;
                    (l > 0 ? t.pos : t.neg) |= uint32_t(1) << p;
                }
                // crossing clauses constrain the block only when exactly-one
                // with at least two literals inside
                if (!t.inside && !(t.kind == TN_CLAUSE_EXACTLY_ONE && inside >= 2)) continue;
                tests.push_back(t);
            }
        const uint64_t cnt = count_block(k, tests);
        if (cnt == 0) return 0;
        bits += std::log2(double(cnt));
    }
    return int32_t(std::min<double>(double(n), std::ceil(bits + 1e-9)));
}

}  // namespace tn
