// Host check of the partition order's bisection on small random graphs:
// with at most 12 vertices every split is tried, so bisect must return a
// cut as light as the lightest split within the balance window found by
// brute force here; with 13 to 24 vertices (graph growing and
// Fiduccia-Mattheyses) the split must lie within the window. In both cases
// the reported cut must be the returned split's. The window restates the
// partition code's rule: side 0 may weigh W/2 -/+ max(heaviest vertex,
// 5 % of W), kept within [1, W - 1]. Prints "ok" at the end; a violation
// exits with status 1.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "graph.hpp"

using namespace tn;

int main() {
    SplitMix gen(12345);
    int bad = 0, exact = 0, checked = 0;
    for (int trial = 0; trial < 3000; ++trial) {
        const int n = 2 + int(gen.below(23));  // 2 .. 24 vertices
        // random edges (weights 1..3) over random vertex weights 1..2
        std::vector<std::vector<std::pair<int32_t, int32_t>>> al(n);
        const int m = int(gen.below(uint32_t(3 * n))) + n - 1;
        for (int e = 0; e < m; ++e) {
            const int32_t a = int32_t(gen.below(uint32_t(n))), b = int32_t(gen.below(uint32_t(n)));
            if (a == b) continue;
            bool dup = false;
            for (auto& pr : al[a]) dup = dup || pr.first == b;
            if (dup) continue;
            const int32_t w = 1 + int32_t(gen.below(3));
            al[a].push_back({b, w});
            al[b].push_back({a, w});
        }
        WGraph g;
        g.n = n;
        g.xadj.assign(n + 1, 0);
        for (int v = 0; v < n; ++v) {
            std::sort(al[v].begin(), al[v].end());
            for (auto& pr : al[v]) {
                g.adj.push_back(pr.first);
                g.ew.push_back(pr.second);
            }
            g.xadj[v + 1] = int32_t(g.adj.size());
            g.vw.push_back(1 + int32_t(gen.below(2)));
        }
        const int64_t W = g.total_vw();
        int64_t maxw = 0;
        for (int32_t w : g.vw) maxw = std::max<int64_t>(maxw, w);
        const int64_t tol = std::max<int64_t>(maxw, (W * 5 + 99) / 100);
        int64_t lo = std::max<int64_t>(1, W / 2 - tol), hi = std::min<int64_t>(W - 1, (W + 1) / 2 + tol);
        if (lo > hi) lo = hi = W / 2;
        auto cut_of = [&](const std::vector<uint8_t>& s) {
            int64_t c = 0;
            for (int v = 0; v < n; ++v)
                for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
                    if (s[v] != s[g.adj[e]]) c += g.ew[e];
            return c / 2;
        };
        auto w0_of = [&](const std::vector<uint8_t>& s) {
            int64_t w = 0;
            for (int v = 0; v < n; ++v)
                if (s[v] == 0) w += g.vw[v];
            return w;
        };
        SplitMix rng(uint64_t(trial) + 1);
        int64_t cut = -1;
        const std::vector<uint8_t> side = bisect(g, rng, &cut);
        if (int(side.size()) != n || cut != cut_of(side)) {
            std::printf("trial %d (n %d): reported cut %lld, split's cut %lld\n", trial, n, (long long)cut,
                        (long long)cut_of(side));
            bad = 1;
            continue;
        }
        // brute force over every split (vertex 0 on side 0; the window is
        // symmetric)
        int64_t best = -1;
        for (uint32_t mask = 0; mask < (uint32_t(1) << (n - 1)) && n <= 12; ++mask) {
            std::vector<uint8_t> s(n, 0);
            for (int v = 1; v < n; ++v) s[v] = uint8_t((mask >> (v - 1)) & 1);
            const int64_t w0 = w0_of(s);
            if (w0 < lo || w0 > hi) continue;
            const int64_t c = cut_of(s);
            if (best < 0 || c < best) best = c;
        }
        const int64_t w0 = w0_of(side);
        const bool within = (w0 >= lo && w0 <= hi) || (W - w0 >= lo && W - w0 <= hi);
        if (n <= 12 && best >= 0) {
            ++exact;
            if (cut != best || !within) {
                std::printf("trial %d (n %d): cut %lld, lightest balanced %lld, side-0 weight %lld in [%lld, %lld]\n",
                            trial, n, (long long)cut, (long long)best, (long long)w0, (long long)lo, (long long)hi);
                bad = 1;
            }
        } else if (n > 12 && !within) {
            std::printf("trial %d (n %d): side-0 weight %lld outside [%lld, %lld]\n", trial, n, (long long)w0,
                        (long long)lo, (long long)hi);
            bad = 1;
        }
        ++checked;
    }
    std::printf("%d graphs, %d against brute force: %s\n", checked, exact, bad ? "MISMATCH" : "ok");
    return bad;
}
