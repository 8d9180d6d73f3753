// Host check of the local reconfiguration of contraction trees: for
// partition orders of a formula read from stdin ("n m", then per clause
// "kind len literals..."), reconfiguring to convergence must give a valid
// plan, no more costly under the cost model, with no larger a largest
// rank, and the same merges when run again. Prints one line per order and
// "ok" at the end; a violation exits with status 1.
#include <cstdio>
#include <limits>
#include <vector>

#include "internal.hpp"
#include "tn.h"

using namespace tn;

int main() {
    int n = 0, m = 0;
    if (std::scanf("%d %d", &n, &m) != 2) return 2;
    std::vector<int32_t> ptr{0}, lits;
    std::vector<uint8_t> kinds;
    for (int c = 0; c < m; ++c) {
        int k = 0, l = 0;
        if (std::scanf("%d %d", &k, &l) != 2) return 2;
        kinds.push_back(uint8_t(k));
        for (int i = 0; i < l; ++i) {
            int x = 0;
            if (std::scanf("%d", &x) != 1) return 2;
            lits.push_back(x);
        }
        ptr.push_back(int32_t(lits.size()));
    }
    tn_formula f{n, m, ptr.data(), lits.data(), kinds.data()};
    Network net;
    if (build_network(&f, net) != TN_OK) return 2;
    const double forever = std::numeric_limits<double>::infinity();
    int bad = 0;
    for (uint64_t seed = 1; seed <= 5; ++seed) {
        const auto merges = order_partition(net, seed);
        Plan before, after;
        if (make_plan(net, merges, TN_ORDER_PARTITION, before) != TN_OK) continue;  // beyond the rank cap
        const auto r1 = refine_order(net, merges, forever);
        const auto r2 = refine_order(net, merges, forever);
        const tn_status st = make_plan(net, r1, TN_ORDER_PARTITION, after);
        const bool ok = st == TN_OK && verify_plan(after) == TN_OK && r1 == r2 &&
                        plan_cost(after) <= plan_cost(before) * (1 + 1e-12) &&
                        after.stats.max_rank <= before.stats.max_rank;
        std::printf("seed %llu: cost %.6g -> %.6g us, rank %d -> %d%s\n", (unsigned long long)seed, plan_cost(before),
                    st == TN_OK ? plan_cost(after) : -1.0, before.stats.max_rank, after.stats.max_rank,
                    ok ? "" : "  VIOLATION");
        bad |= !ok;
    }
    std::printf(bad ? "MISMATCH\n" : "ok\n");
    return bad;
}
