// Host check of the judge's plan sketches: for the merges of partition and
// community orders of a formula read from stdin ("n m", then per clause
// "kind len literals..."), sketch_plan must give the status, predicted cost
// (to the last bit), largest rank and step count that make_plan gives, and
// both must reject the same broken merge lists. Prints one line per case
// and "ok" at the end; any mismatch exits with status 1.
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "tn.h"

using namespace tn;
using Merges = std::vector<std::pair<int32_t, int32_t>>;

static int compare(const Network& net, const Merges& m, const char* what) {
    Plan full, sk;
    const tn_status a = make_plan(net, m, TN_ORDER_PARTITION, full);
    const tn_status b = sketch_plan(net, m, TN_ORDER_PARTITION, sk);
    if (a != b) {
        std::printf("%s: status %d (full) against %d (sketch)\n", what, int(a), int(b));
        return 1;
    }
    if (a != TN_OK) {
        std::printf("%s: both %d\n", what, int(a));
        return 0;
    }
    const double cf = plan_cost(full), cs = plan_cost(sk);
    if (std::memcmp(&cf, &cs, sizeof cf) != 0 || full.stats.max_rank != sk.stats.max_rank ||
        full.stats.n_steps != sk.stats.n_steps || full.root != sk.root || full.stats.log2_cost != sk.stats.log2_cost) {
        std::printf("%s: cost %.17g against %.17g, rank %d against %d, steps %d against %d\n", what, cf, cs,
                    full.stats.max_rank, sk.stats.max_rank, full.stats.n_steps, sk.stats.n_steps);
        return 1;
    }
    std::printf("%s: cost %.6g us, rank %d\n", what, cf, full.stats.max_rank);
    return 0;
}

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
    int bad = 0;
    char what[64];
    for (uint64_t seed = 1; seed <= 6; ++seed) {
        std::snprintf(what, sizeof what, "partition seed %llu", (unsigned long long)seed);
        bad |= compare(net, order_partition(net, seed), what);
    }
    bad |= compare(net, order_community(net), "community");
    // broken merge lists: a merge of a consumed tensor, an id out of range,
    // a merge left out (two tensors alive at the end)
    Merges g = order_partition(net, 1);
    if (g.size() >= 2) {
        Merges x = g;
        x[1] = x[0];
        bad |= compare(net, x, "repeated merge");
        Merges y = g;
        y.back().first = int32_t(net.t.size() + g.size());
        bad |= compare(net, y, "id out of range");
        Merges z = g;
        z.pop_back();
        bad |= compare(net, z, "merge left out");
    }
    std::printf(bad ? "MISMATCH\n" : "ok\n");
    return bad;
}
