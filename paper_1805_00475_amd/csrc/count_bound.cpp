// Upper bound on the count of a boolean formula, used to size the residue
// system: the count is recovered from its residues modulo moduli whose
// product exceeds the bound (Sec. 2.1, the count as the full trace; Sec. 3.2
// on exactness), so a tighter bound means fewer residue planes.
//
// The count is the sum over assignments of the product of the clause tables
// (0/1 valued). Variables are eliminated one at a time (fewest neighbours
// first). When the tables that hold a variable v span at most ib other
// variables, they are multiplied and v is summed out, as in exact
// elimination. Otherwise they are split into mini-buckets of at most ib
// other variables each: v is summed out of the product of the first and
// maximised out of the product of each other one. For non-negative tables
//   sum_v prod_j P_j(v, .) <= sum_v P_1(v, .) * prod_{j>1} max_v P_j(v, .),
// so the result bounds the count from above. Clauses that use a variable
// twice are left out (every table is at most 1, so dropping one only raises
// the sum), and an empty clause makes the count 0.
//
// A tighter variant (count_bound_bits_tight) bounds every mini-bucket by
// Hoelder's inequality instead: with k mini-buckets,
//   sum_v prod_j P_j(v, .) <= prod_j (sum_v P_j(v, .)^k)^(1/k),
// one k-norm per mini-bucket (k = 1 is the exact sum); it takes
// mini-buckets of up to 17 other variables and eliminates by least fill
// among the 16 variables of fewest neighbours. It costs about four times as
// much (about 40 ms at n = 300) and saves one residue plane on the largest
// configurations (1-in-3 n = 300: 85 bits against 93; the norms alone at
// 15 other variables give 90).
//
// Tables hold doubles; every new table is scaled by a power of two (exact)
// so that its largest entry lies in [1, 2), the scale going into a running
// log2 sum. Entries are sums, products and maxima of non-negative numbers,
// so each carries a relative rounding error below (k + 2) 2^-53 per
// elimination it went through (k tables per bucket); over at most n
// eliminations this stays far below the margin of 1e-6 added in log2.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <set>
#include <vector>

#include "internal.hpp"

namespace tn {

namespace {

// other variables of a mini-bucket: 15 (tables of up to 2^16 entries) from
// kBigFrom variables on, 10 below, where the bound costs about 1.5 ms
// instead of about 10 (vertex cover n = 120: 80 bits against 78)
constexpr int kIBoundBig = 15, kIBoundSmall = 10, kBigFrom = 160;
// the tighter variant: mini-buckets of up to 17 other variables (tables of
// up to 2^18 entries), least fill among the 16 variables of fewest
// neighbours (at n = 300: 85 bits against 88 with 16 others, 86 with 8
// candidates)
constexpr int kIBoundTight = 17, kFillCands = 16;

struct Table {
    std::vector<int32_t> vars;  // bit i of an index is the value of vars[i]
    std::vector<double> t;
    bool alive = true;
};

// multiply `src` (over its vars) into `dst`, a table over `scope` (a
// superset of at most 24 variables), bit j of an index of dst being
// scope[j]; the index into src is a bit selection, looked up per byte
void accumulate(const Table& src, const std::vector<int32_t>& scope, std::vector<double>& dst) {
    uint32_t look[3][256] = {};
    for (size_t i = 0; i < src.vars.size(); ++i) {
        const int at = int(std::find(scope.begin(), scope.end(), src.vars[i]) - scope.begin());
        for (uint32_t b = 0; b < 256; ++b)
            if ((b >> (at % 8)) & 1) look[at / 8][b] |= uint32_t(1) << i;
    }
    for (size_t a = 0; a < dst.size(); ++a)
        dst[a] *= src.t[look[0][a & 255] | look[1][(a >> 8) & 255] | look[2][(a >> 16) & 255]];
}

}  // namespace

// The elimination: mini-buckets of at most ib other variables, Hoelder
// norms (weighted) or one sum and maxima, the next variable by fewest
// neighbours or, with fill_cands > 0, by least fill among the fill_cands
// variables of fewest neighbours (ties: fewer neighbours, lower index).
int32_t count_bound_bits_with(const tn_formula* f, int ib, bool weighted, int fill_cands,
                              const std::atomic<bool>* cancel) {
    const int32_t n = f->n_vars, m = f->n_clauses;
    std::vector<Table> tabs;
    std::vector<std::vector<int32_t>> holds(static_cast<size_t>(n));  // tables holding each variable
    for (int32_t c = 0; c < m; ++c) {
        const int32_t b = f->clause_ptr[c], e = f->clause_ptr[c + 1];
        if (b == e) return 0;  // an empty clause: the count is 0
        Table x;
        bool usable = true;
        for (int32_t i = b; i < e; ++i) {
            const int32_t v = std::abs(f->lits[i]) - 1;
            if (std::find(x.vars.begin(), x.vars.end(), v) != x.vars.end()) usable = false;
            x.vars.push_back(v);
        }
        if (!usable) continue;
        const size_t w = x.vars.size();
        x.t.resize(size_t(1) << w);
        for (size_t a = 0; a < x.t.size(); ++a) {
            int ones = 0;
            for (size_t i = 0; i < w; ++i) ones += int(((a >> i) & 1) ^ (f->lits[b + int32_t(i)] < 0 ? 1 : 0));
            const bool ok = f->kinds[c] == TN_CLAUSE_OR ? ones >= 1
                            : f->kinds[c] == TN_CLAUSE_EXACTLY_ONE ? ones == 1
                                                                  : (ones & 1) == 1;
            x.t[a] = ok ? 1.0 : 0.0;
        }
        for (int32_t v : x.vars) holds[size_t(v)].push_back(int32_t(tabs.size()));
        tabs.push_back(std::move(x));
    }
    std::vector<std::set<int32_t>> adj(static_cast<size_t>(n));
    // the same adjacency as bit rows, kept for the least-fill order
    const size_t words = size_t(n + 63) / 64;
    std::vector<uint64_t> rows(fill_cands > 0 ? size_t(n) * words : 0, 0);
    auto link = [&](int32_t u, int32_t y) {
        adj[size_t(u)].insert(y);
        if (fill_cands > 0) rows[size_t(u) * words + size_t(y) / 64] |= uint64_t(1) << (y % 64);
    };
    for (const Table& x : tabs)
        for (int32_t u : x.vars)
            for (int32_t y : x.vars)
                if (y != u) link(u, y);
    std::vector<char> alive(static_cast<size_t>(n), 1);
    double bits = 0;
    for (int32_t step = 0; step < n; ++step) {
        if (cancel && cancel->load(std::memory_order_relaxed)) return -1;
        int32_t v = -1;
        size_t deg = 0;
        if (fill_cands > 0) {
            std::vector<std::pair<size_t, int32_t>> cands;
            for (int32_t u = 0; u < n; ++u)
                if (alive[size_t(u)]) cands.push_back({adj[size_t(u)].size(), u});
            if (int(cands.size()) > fill_cands) {
                std::nth_element(cands.begin(), cands.begin() + fill_cands, cands.end());
                cands.resize(size_t(fill_cands));
            }
            std::sort(cands.begin(), cands.end());
            long best_fill = -1;
            for (const auto& cu : cands) {
                // pairs of neighbours not yet adjacent: each neighbour's
                // non-neighbours among the others, counted from both ends
                const uint64_t* ru = rows.data() + size_t(cu.second) * words;
                long fill = 0;
                for (int32_t a : adj[size_t(cu.second)]) {
                    const uint64_t* ra = rows.data() + size_t(a) * words;
                    for (size_t w = 0; w < words; ++w) fill += __builtin_popcountll(ru[w] & ~ra[w]);
                    --fill;  // a itself
                }
                fill /= 2;
                if (best_fill < 0 || fill < best_fill) {
                    best_fill = fill;
                    v = cu.second;
                    deg = cu.first;
                }
            }
        } else {
            for (int32_t u = 0; u < n; ++u)
                if (alive[size_t(u)] && (v < 0 || adj[size_t(u)].size() < deg)) {
                    v = u;
                    deg = adj[size_t(u)].size();
                }
        }
        alive[size_t(v)] = 0;
        for (int32_t y : adj[size_t(v)]) {
            adj[size_t(y)].erase(v);
            if (fill_cands > 0) rows[size_t(y) * words + size_t(v) / 64] &= ~(uint64_t(1) << (v % 64));
        }
        std::vector<int32_t> bucket;
        for (int32_t id : holds[size_t(v)])
            if (tabs[size_t(id)].alive) bucket.push_back(id);
        if (bucket.empty()) {  // in no table: both values count
            bits += 1.0;
            continue;
        }
        // mini-buckets, larger tables first, each into the first whose scope
        // stays within v and ib others
        std::stable_sort(bucket.begin(), bucket.end(), [&](int32_t a, int32_t b) {
            return tabs[size_t(a)].vars.size() > tabs[size_t(b)].vars.size();
        });
        std::vector<std::vector<int32_t>> mb, mbscope;
        for (int32_t id : bucket) {
            tabs[size_t(id)].alive = false;
            const auto& vs = tabs[size_t(id)].vars;
            bool placed = false;
            for (size_t j = 0; j < mb.size() && !placed; ++j) {
                std::vector<int32_t> u = mbscope[j];
                for (int32_t y : vs)
                    if (std::find(u.begin(), u.end(), y) == u.end()) u.push_back(y);
                if (int(u.size()) <= ib + 1) {
                    mbscope[j] = u;
                    mb[j].push_back(id);
                    placed = true;
                }
            }
            if (!placed) {
                mb.push_back({id});
                mbscope.push_back(vs);
            }
        }
        for (size_t j = 0; j < mb.size(); ++j) {
            // v first, then the others
            std::vector<int32_t> scope{v};
            for (int32_t y : mbscope[j])
                if (y != v) scope.push_back(y);
            std::vector<double> prod(size_t(1) << scope.size(), 1.0);
            for (int32_t id : mb[j]) accumulate(tabs[size_t(id)], scope, prod);
            Table out;
            out.vars.assign(scope.begin() + 1, scope.end());
            out.t.resize(prod.size() / 2);
            double mx = 0;
            const double k = double(mb.size());
            for (size_t a = 0; a < out.t.size(); ++a) {
                const double lo = prod[2 * a], hi = prod[2 * a + 1];
                if (!weighted || mb.size() == 1) {
                    out.t[a] = j == 0 ? lo + hi : std::max(lo, hi);
                } else {
                    // (lo^k + hi^k)^(1/k), factored by the larger so that
                    // nothing overflows; an underflowing ratio^k loses a
                    // relative error below 2^-1000
                    const double big = std::max(lo, hi), small = std::min(lo, hi);
                    out.t[a] = big > 0 ? big * std::pow(1.0 + std::pow(small / big, k), 1.0 / k) : 0.0;
                }
                mx = std::max(mx, out.t[a]);
            }
            if (mx <= 0) return 0;  // no assignment passes: the count is 0
            int e = 0;
            (void)std::frexp(mx, &e);  // mx in [2^(e-1), 2^e)
            for (double& x : out.t) x = std::ldexp(x, 1 - e);
            bits += double(e - 1);
            if (out.vars.empty()) {
                bits += std::log2(out.t[0]);
                continue;
            }
            for (int32_t u : out.vars) {
                holds[size_t(u)].push_back(int32_t(tabs.size()));
                for (int32_t y : out.vars)
                    if (y != u) link(u, y);
            }
            tabs.push_back(std::move(out));
        }
    }
    return int32_t(std::min<double>(double(n), std::ceil(bits + 1e-6)));
}

double disjoint_clause_bound_bits(const tn_formula* f) {
    // The formula restricted to clauses taken greedily in order while they
    // share no variable with those taken (and repeat none): its count,
    // 2^(n - sum |c|) prod sat(c), is at least the formula's, since leaving
    // clauses out only adds solutions.
    std::vector<char> used(size_t(std::max(0, f->n_vars)), 0);
    double bits = double(f->n_vars);
    for (int32_t c = 0; c < f->n_clauses; ++c) {
        const int32_t b = f->clause_ptr[c], e = f->clause_ptr[c + 1];
        if (b == e) return 0.0;  // an empty clause: no solution
        bool free = true;
        for (int32_t i = b; i < e && free; ++i) {
            const int32_t v = std::abs(f->lits[i]) - 1;
            free = !used[size_t(v)];
            for (int32_t j = b; j < i && free; ++j) free = std::abs(f->lits[j]) - 1 != v;
        }
        if (!free) continue;
        const int k = e - b;
        const double sat = f->kinds[c] == TN_CLAUSE_OR ? std::ldexp(1.0, k) - 1.0
                           : f->kinds[c] == TN_CLAUSE_EXACTLY_ONE ? double(k)
                                                                 : std::ldexp(1.0, k - 1);
        bits += std::log2(sat) - double(k);
        for (int32_t i = b; i < e; ++i) used[size_t(std::abs(f->lits[i]) - 1)] = 1;
    }
    return bits;
}

int32_t count_bound_bits(const tn_formula* f) {
    return count_bound_bits_with(f, f->n_vars >= kBigFrom ? kIBoundBig : kIBoundSmall, false, 0);
}

int32_t count_bound_bits_tight(const tn_formula* f, const std::atomic<bool>* cancel) {
    return count_bound_bits_with(f, kIBoundTight, true, kFillCands, cancel);
}

}  // namespace tn
