// Host check of the count bounds (and the quick disjoint-clause bound) on
// random small formulas: OR,
// exactly-one and parity clauses of 1 to 4 literals with negations and
// repeats, 4 to 20 variables. Every bound b (the library's two, and the
// same elimination with mini-buckets of 1 to 4 other variables, with one
// sum and maxima or with Hoelder norms, by fewest neighbours or least fill,
// so that buckets split often) must satisfy count <= 2^b, the count found
// by enumerating every assignment here. Prints "ok" at the end; a
// violation exits with status 1.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "graph.hpp"
#include "internal.hpp"

using namespace tn;

int main() {
    SplitMix gen(2024);
    int bad = 0, tighter = 0, looser = 0, cases = 0;
    for (int trial = 0; trial < 600; ++trial) {
        const int n = 4 + int(gen.below(17));
        const int m = 1 + int(gen.below(uint32_t(2 * n)));
        std::vector<int32_t> ptr{0}, lits;
        std::vector<uint8_t> kinds;
        for (int c = 0; c < m; ++c) {
            const int len = 1 + int(gen.below(4));
            for (int i = 0; i < len; ++i) {
                const int32_t v = 1 + int32_t(gen.below(uint32_t(n)));
                lits.push_back(gen.below(2) ? v : -v);
            }
            ptr.push_back(int32_t(lits.size()));
            kinds.push_back(uint8_t(gen.below(3)));  // OR, exactly-one, parity
        }
        tn_formula f{n, m, ptr.data(), lits.data(), kinds.data()};
        uint64_t count = 0;
        for (uint64_t x = 0; x < (uint64_t(1) << n); ++x) {
            bool ok = true;
            for (int c = 0; c < m && ok; ++c) {
                int ones = 0;
                for (int32_t i = ptr[c]; i < ptr[c + 1]; ++i) {
                    const int32_t l = lits[size_t(i)];
                    ones += int(((x >> (std::abs(l) - 1)) & 1) ^ (l < 0 ? 1u : 0u));
                }
                ok = kinds[size_t(c)] == TN_CLAUSE_OR ? ones >= 1
                     : kinds[size_t(c)] == TN_CLAUSE_EXACTLY_ONE ? ones == 1
                                                                  : (ones & 1) == 1;
            }
            count += ok;
        }
        const double need = count ? std::log2(double(count)) : -1.0;
        const double quick = disjoint_clause_bound_bits(&f);
        if (quick < need - 1e-9) {
            std::printf("trial %d (n %d, m %d): count %llu, disjoint-clause bound %.3f bits\n", trial, n, m,
                        (unsigned long long)count, quick);
            bad = 1;
        }
        std::vector<int32_t> bs{count_bound_bits(&f), count_bound_bits_tight(&f)};
        for (int ib = 1; ib <= 4; ++ib)
            for (int w = 0; w < 2; ++w)
                for (int fc : {0, 4}) bs.push_back(count_bound_bits_with(&f, ib, w == 1, fc));
        ++cases;
        // small mini-buckets, max-based against Hoelder (same order)
        for (int ib = 1; ib <= 4; ++ib) {
            const int32_t mx = bs[size_t(2 + (ib - 1) * 4)], ho = bs[size_t(2 + (ib - 1) * 4 + 2)];
            tighter += ho < mx;
            looser += ho > mx;
        }
        for (size_t i = 0; i < bs.size(); ++i)
            if (double(bs[i]) < need - 1e-9) {
                std::printf("trial %d (n %d, m %d): count %llu, bound %zu gives %d bits\n", trial, n, m,
                            (unsigned long long)count, i, bs[i]);
                bad = 1;
            }
    }
    std::printf("%d formulas (Hoelder norms lower than sum and maxima on %d bounds, higher on %d): %s\n", cases, tighter,
                looser, bad ? "MISMATCH" : "ok");
    return bad;
}
