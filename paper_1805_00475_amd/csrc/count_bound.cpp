// Upper bound on the count of a boolean formula, used to size the residue
// system: the count is recovered from its residues modulo moduli whose
// product exceeds the bound (Sec. 2.1, the count as the full trace; Sec. 3.2
// on exactness), so a tighter bound means fewer residue planes.
//
// The variables are split into blocks. For an assignment x every clause
// value is 0 or 1, and a satisfied clause passes these tests on the
// restriction of x to any block B: a clause lying inside B is satisfied
// there, and an exactly-one clause that only partly lies in B has at most one
// true literal there. Hence the product of the clause values is at most the
// product over blocks of the indicator that x|B passes every test of B, and
// summing over x, the count is at most the product over blocks of the number
// of assignments of B passing its tests. Clauses that use a variable twice
// are left out of the tests (a relaxation), and an empty clause makes the
// count 0.
//
// Blocks are grown greedily around the variables in most clauses, adding the
// neighbour that completes most clauses. A block of at most 20 variables is
// counted by bit slicing (64 assignments of its six lowest variables per
// machine word); a larger one by variable elimination over its tests in
// double precision (every table entry is a sum of products of 0/1 values;
// with at most a few thousand roundings along any path, each of relative
// size below 2^-53, the result is within a relative 1e-12 of the exact
// count, and a margin of 1e-6 in log2 covers it). A block whose elimination
// would need a table over more than kMaxWidth variables is split again into
// blocks of half its size. Large formulas (from kBigFrom variables) use blocks of up to
// kBigBlock variables, smaller ones blocks of 16, whose cost is a few
// milliseconds at most.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <vector>

#include "internal.hpp"

namespace tn {

namespace {

constexpr int kSmallBlock = 16;
constexpr int kBigBlock = 96;
constexpr int kBigFrom = 160;
constexpr int kSliceMax = 20;
constexpr int kMaxWidth = 20;

struct Lit {
    int32_t var;  // block-local
    bool neg;
};

struct Test {
    int kind;     // TN_CLAUSE_*
    bool inside;  // every literal in the block (else: exactly-one, at most one true here)
    std::vector<Lit> lits;
};

struct Formula {
    const tn_formula* f;
    std::vector<std::vector<int32_t>> cl_of;  // usable clauses of each variable
    int32_t var(int64_t i) const { return std::abs(f->lits[i]) - 1; }
};

// Blocks of at most B variables among those with block_of = -1 (others are
// placed already), grown from the unplaced variable in most clauses; new
// block ids start at `first`.
std::vector<std::vector<int32_t>> grow_blocks(const Formula& F, std::vector<int32_t>& block_of,
                                              const std::vector<int32_t>& vars, int B, int32_t first) {
    std::vector<int32_t> order(vars);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return F.cl_of[size_t(a)].size() > F.cl_of[size_t(b)].size();
    });
    std::vector<std::vector<int32_t>> blocks;
    for (int32_t s : order) {
        if (block_of[size_t(s)] != -1) continue;
        const int32_t id = first + int32_t(blocks.size());
        blocks.push_back({s});
        block_of[size_t(s)] = id;
        std::vector<int32_t>& blk = blocks.back();
        while (int(blk.size()) < B) {
            int32_t best = -1;
            double bs = -1;
            for (size_t bi = 0; bi < blk.size(); ++bi)
                for (int32_t c : F.cl_of[size_t(blk[bi])])
                    for (int32_t i = F.f->clause_ptr[c]; i < F.f->clause_ptr[c + 1]; ++i) {
                        const int32_t u = F.var(i);
                        if (block_of[size_t(u)] != -1) continue;
                        double sc = 0;
                        for (int32_t c2 : F.cl_of[size_t(u)]) {
                            bool all = true, touch = false;
                            for (int32_t j = F.f->clause_ptr[c2]; j < F.f->clause_ptr[c2 + 1]; ++j) {
                                const int32_t w = F.var(j);
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
    return blocks;
}

// the tests of one block (variables numbered by their place in blk)
std::vector<Test> block_tests(const Formula& F, const std::vector<int32_t>& block_of,
                              const std::vector<int32_t>& blk) {
    std::vector<Test> tests;
    std::vector<int32_t> seen;
    const int32_t id = block_of[size_t(blk[0])];
    for (size_t j = 0; j < blk.size(); ++j)
        for (int32_t c : F.cl_of[size_t(blk[j])]) {
            if (std::find(seen.begin(), seen.end(), c) != seen.end()) continue;
            seen.push_back(c);
            Test t{F.f->kinds[c], true, {}};
            for (int32_t i = F.f->clause_ptr[c]; i < F.f->clause_ptr[c + 1]; ++i) {
                const int32_t w = F.var(i);
                if (block_of[size_t(w)] != id) {
                    t.inside = false;
                    continue;
                }
                const int32_t p = int32_t(std::find(blk.begin(), blk.end(), w) - blk.begin());
                t.lits.push_back({p, F.f->lits[i] < 0});
            }
            if (!t.inside && !(t.kind == TN_CLAUSE_EXACTLY_ONE && t.lits.size() >= 2)) continue;
            tests.push_back(std::move(t));
        }
    return tests;
}

bool passes(const Test& t, int ones) {
    if (t.kind == TN_CLAUSE_OR) return ones >= 1;
    if (t.kind == TN_CLAUSE_EXACTLY_ONE) return t.inside ? ones == 1 : ones <= 1;
    return ones & 1;  // parity
}

// lane patterns of the six lowest block variables over 64 assignments
constexpr uint64_t kLane[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                               0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};

uint64_t count_sliced(int k, const std::vector<Test>& tests) {
    const int low = std::min(k, 6);
    const uint64_t lanes = low == 6 ? ~uint64_t(0) : ((uint64_t(1) << (1 << low)) - 1);
    uint64_t word[kSliceMax];
    uint64_t total = 0;
    for (uint64_t h = 0; h < (uint64_t(1) << (k - low)); ++h) {
        for (int j = 0; j < k; ++j) word[j] = j < 6 ? kLane[j] : (((h >> (j - 6)) & 1) ? ~uint64_t(0) : 0);
        uint64_t ok = lanes;
        for (const Test& t : tests) {
            uint64_t one = 0, two = 0, any = 0;  // odd count, two or more, at least one
            for (const Lit& l : t.lits) {
                const uint64_t x = l.neg ? ~word[l.var] : word[l.var];
                two |= one & x;
                one ^= x;
                any |= x;
            }
            if (t.kind == TN_CLAUSE_OR) ok &= any;
            else if (t.kind == TN_CLAUSE_EXACTLY_ONE) ok &= t.inside ? (one & ~two) : ~two;
            else ok &= one;
            if (!ok) break;
        }
        total += uint64_t(__builtin_popcountll(ok));
    }
    return total;
}

struct Table {
    std::vector<int32_t> vars;  // bit i of an index is the value of vars[i]
    std::vector<double> t;
};

// log2 of the block count by variable elimination (min-degree order), or NaN
// when a table would span more than kMaxWidth variables
double log2_eliminated(int k, const std::vector<Test>& tests) {
    std::vector<Table> tabs;
    for (const Test& t : tests) {
        Table x;
        for (const Lit& l : t.lits) x.vars.push_back(l.var);
        const size_t w = x.vars.size();
        x.t.resize(size_t(1) << w);
        for (size_t a = 0; a < x.t.size(); ++a) {
            int ones = 0;
            for (size_t i = 0; i < w; ++i) ones += int(((a >> i) & 1) ^ (t.lits[i].neg ? 1 : 0));
            x.t[a] = passes(t, ones) ? 1.0 : 0.0;
        }
        tabs.push_back(std::move(x));
    }
    std::vector<char> alive(size_t(k), 1);
    double log2sum = 0;
    for (int step = 0; step < k; ++step) {
        // the variable with the fewest neighbours (ties: lowest index)
        int v = -1;
        size_t deg = 0;
        for (int u = 0; u < k; ++u) {
            if (!alive[size_t(u)]) continue;
            std::vector<int32_t> nb;
            for (const Table& x : tabs)
                if (std::find(x.vars.begin(), x.vars.end(), u) != x.vars.end())
                    for (int32_t y : x.vars)
                        if (y != u && std::find(nb.begin(), nb.end(), y) == nb.end()) nb.push_back(y);
            if (v < 0 || nb.size() < deg) {
                v = u;
                deg = nb.size();
            }
        }
        alive[size_t(v)] = 0;
        std::vector<Table> bucket, rest;
        for (Table& x : tabs)
            (std::find(x.vars.begin(), x.vars.end(), v) != x.vars.end() ? bucket : rest).push_back(std::move(x));
        if (bucket.empty()) {  // a variable in no test: both values pass
            log2sum += 1.0;
            tabs = std::move(rest);
            continue;
        }
        std::vector<int32_t> scope;
        for (const Table& x : bucket)
            for (int32_t y : x.vars)
                if (y != v && std::find(scope.begin(), scope.end(), y) == scope.end()) scope.push_back(y);
        if (int(scope.size()) + 1 > kMaxWidth) return std::nan("");
        // position of each table variable in (v, scope...)
        std::vector<std::vector<int>> where(bucket.size());
        for (size_t b = 0; b < bucket.size(); ++b)
            for (int32_t y : bucket[b].vars)
                where[b].push_back(y == v ? 0 : 1 + int(std::find(scope.begin(), scope.end(), y) - scope.begin()));
        Table out;
        out.vars = scope;
        out.t.assign(size_t(1) << scope.size(), 0.0);
        for (size_t a = 0; a < out.t.size(); ++a) {
            double s = 0;
            for (size_t xv = 0; xv < 2; ++xv) {
                const size_t full = xv | (a << 1);
                double p = 1;
                for (size_t b = 0; b < bucket.size() && p != 0; ++b) {
                    size_t idx = 0;
                    for (size_t i = 0; i < where[b].size(); ++i) idx |= ((full >> where[b][i]) & 1) << i;
                    p *= bucket[b].t[idx];
                }
                s += p;
            }
            out.t[a] = s;
        }
        rest.push_back(std::move(out));
        tabs = std::move(rest);
        // constant tables go into the running sum
        for (size_t i = 0; i < tabs.size();) {
            if (tabs[i].vars.empty()) {
                if (tabs[i].t[0] <= 0) return -INFINITY;
                log2sum += std::log2(tabs[i].t[0]);
                tabs.erase(tabs.begin() + long(i));
            } else {
                ++i;
            }
        }
    }
    return log2sum;
}

}  // namespace

int32_t count_bound_bits(const tn_formula* f) {
    const int32_t n = f->n_vars, m = f->n_clauses;
    Formula F{f, std::vector<std::vector<int32_t>>(static_cast<size_t>(n))};
    for (int32_t c = 0; c < m; ++c) {
        const int32_t b = f->clause_ptr[c], e = f->clause_ptr[c + 1];
        if (b == e) return 0;  // an empty clause: the count is 0
        bool usable = true;
        for (int32_t i = b; i < e && usable; ++i)
            for (int32_t j = b; j < i; ++j)
                if (F.var(i) == F.var(j)) usable = false;
        if (!usable) continue;
        for (int32_t i = b; i < e; ++i) F.cl_of[size_t(F.var(i))].push_back(c);
    }
    std::vector<int32_t> block_of(static_cast<size_t>(n), -1), all(static_cast<size_t>(n));
    for (int32_t v = 0; v < n; ++v) all[size_t(v)] = v;
    int32_t next_id = 0;
    bool zero = false;
    // bound over the variables `vars` (unplaced) in blocks of at most B; a
    // block too wide to eliminate is split again into blocks of half the size
    std::function<double(const std::vector<int32_t>&, int)> bound = [&](const std::vector<int32_t>& vars, int B) {
        auto blocks = grow_blocks(F, block_of, vars, B, next_id);
        next_id += int32_t(blocks.size());
        double bits = 0;
        for (const auto& blk : blocks) {
            const int k = int(blk.size());
            const auto tests = block_tests(F, block_of, blk);
            if (k <= kSliceMax) {
                const uint64_t cnt = count_sliced(k, tests);
                if (cnt == 0) zero = true;
                else bits += std::log2(double(cnt));
                continue;
            }
            const double lb = log2_eliminated(k, tests);
            if (lb == -INFINITY) {
                zero = true;
            } else if (!std::isnan(lb)) {
                bits += lb + 1e-6;
            } else {
                for (int32_t v : blk) block_of[size_t(v)] = -1;
                bits += bound(blk, std::max(kSmallBlock, B / 2));
            }
        }
        return bits;
    };
    const double bits = bound(all, n >= kBigFrom ? kBigBlock : kSmallBlock);
    if (zero) return 0;
    return int32_t(std::min<double>(double(n), std::ceil(bits + 1e-9)));
}

}  // namespace tn
