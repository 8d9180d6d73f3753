// tensor-greedy order (Sec. 3.1.1): among all pairs of tensors that share
// at least one bond, contract the pair whose result has the smallest rank,
// and repeat until the network is one tensor. The paper fixes only "smallest
// rank"; ties go to the pair that removes the most indices (smallest
// rC - rA - rB), then to the smallest (lower id, higher id).
//
// Also holds the live-tensor graph shared by the orders and the absorption
// pre-pass used by the hierarchical orders.
#include <algorithm>
#include <queue>
#include <tuple>

#include "graph.hpp"
#include "internal.hpp"

namespace tn {

void LiveGraph::init(const Network& net) {
    const int32_t n = int32_t(net.t.size());
    alive.assign(n, 1);
    rank.resize(n);
    nb.assign(n, {});
    bonds.assign(n, {});
    for (int32_t i = 0; i < n; ++i) {
        rank[i] = int32_t(net.t[i].bonds.size());
        bonds[i] = net.t[i].bonds;
        std::sort(bonds[i].begin(), bonds[i].end());
    }
    for (const auto& e : net.bond_end) {
        add_count(e[0], e[1], 1);
        add_count(e[1], e[0], 1);
    }
    next_id = n;
    n_alive = n;
}

void LiveGraph::add_count(int32_t u, int32_t v, int32_t c) {
    auto& m = nb[u];
    for (auto& pr : m)
        if (pr.first == v) {
            pr.second += c;
            return;
        }
    m.push_back({v, c});
}

int32_t LiveGraph::shared(int32_t u, int32_t v) const {
    for (const auto& pr : nb[u])
        if (pr.first == v) return pr.second;
    return 0;
}

int32_t LiveGraph::merge(int32_t a, int32_t b) {
    const int32_t c = next_id++;
    const int32_t s = shared(a, b);
    alive.push_back(1);
    rank.push_back(rank[a] + rank[b] - 2 * s);
    nb.push_back({});
    bonds.push_back({});
    std::vector<int32_t> sd;
    std::set_symmetric_difference(bonds[a].begin(), bonds[a].end(), bonds[b].begin(), bonds[b].end(),
                                  std::back_inserter(sd));
    bonds[c] = std::move(sd);
    for (int32_t x : {a, b}) {
        for (const auto& pr : nb[x]) {
            if (pr.first == a || pr.first == b) continue;
            add_count(c, pr.first, pr.second);
            auto& m = nb[pr.first];
            m.erase(std::remove_if(m.begin(), m.end(),
                                   [&](const std::pair<int32_t, int32_t>& q) { return q.first == a || q.first == b; }),
                    m.end());
        }
    }
    for (const auto& pr : nb[c]) nb[pr.first].push_back({c, pr.second});
    alive[a] = alive[b] = 0;
    nb[a].clear();
    nb[b].clear();
    n_alive -= 1;
    return c;
}

void LiveGraph::close_scalars(std::vector<std::pair<int32_t, int32_t>>& merges) {
    // whatever is left has no bonds (each component reduced to a scalar):
    // multiply the scalars together in id order
    std::vector<int32_t> left;
    for (int32_t i = 0; i < int32_t(alive.size()); ++i)
        if (alive[i]) left.push_back(i);
    while (left.size() > 1) {
        int32_t a = left[0], b = left[1];
        int32_t c = merge(a, b);
        merges.push_back({a, b});
        left.erase(left.begin(), left.begin() + 2);
        left.insert(left.begin(), c);
    }
}

std::vector<std::pair<int32_t, int32_t>> order_greedy(const Network& net) {
    LiveGraph g;
    g.init(net);
    std::vector<std::pair<int32_t, int32_t>> merges;
    using Key = std::tuple<int32_t, int32_t, int32_t, int32_t>;  // rC, rC-rA-rB, lo, hi
    std::priority_queue<Key, std::vector<Key>, std::greater<Key>> heap;
    auto push = [&](int32_t u, int32_t v) {
        int32_t s = g.shared(u, v);
        if (s <= 0) return;
        int32_t rc = g.rank[u] + g.rank[v] - 2 * s;
        heap.push(Key{rc, rc - g.rank[u] - g.rank[v], std::min(u, v), std::max(u, v)});
    };
    for (int32_t u = 0; u < int32_t(g.nb.size()); ++u)
        for (const auto& pr : g.nb[u])
            if (u < pr.first) push(u, pr.first);
    while (!heap.empty()) {
        Key k = heap.top();
        heap.pop();
        int32_t u = std::get<2>(k), v = std::get<3>(k);
        if (!g.alive[u] || !g.alive[v]) continue;
        int32_t c = g.merge(u, v);
        merges.push_back({u, v});
        for (const auto& pr : g.nb[c]) push(c, pr.first);
    }
    g.close_scalars(merges);
    return merges;
}

Reduced absorb_small(const Network& net) {
    LiveGraph g;
    g.init(net);
    Reduced r;
    std::vector<int32_t> work;
    for (int32_t i = 0; i < int32_t(net.t.size()); ++i) work.push_back(i);
    // repeatedly absorb any live tensor of rank <= 2 that still has a
    // neighbour into the neighbour it shares most bonds with (lowest id on
    // ties); the result's rank is at most the neighbour's rank
    size_t head = 0;
    while (head < work.size()) {
        int32_t t = work[head++];
        if (!g.alive[t] || g.rank[t] > 2 || g.nb[t].empty()) continue;
        int32_t best = -1, bs = -1;
        for (const auto& pr : g.nb[t])
            if (pr.second > bs || (pr.second == bs && pr.first < best)) {
                best = pr.first;
                bs = pr.second;
            }
        int32_t c = g.merge(std::min(t, best), std::max(t, best));
        r.merges.push_back({std::min(t, best), std::max(t, best)});
        work.push_back(c);
    }
    for (int32_t i = 0; i < int32_t(g.alive.size()); ++i)
        if (g.alive[i]) {
            r.id.push_back(i);
            r.bonds.push_back(g.bonds[i]);
        }
    r.next_id = g.next_id;
    return r;
}

}  // namespace tn
