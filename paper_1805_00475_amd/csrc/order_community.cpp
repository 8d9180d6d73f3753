// tensor-GN order (Sec. 3.1.1): the Girvan-Newman divisive community
// detection -- repeatedly remove the edge of highest betweenness (the
// number of shortest paths through it) -- used like a separator hierarchy.
// Every removal that disconnects a community splits it in two; the split
// tree, read bottom-up (post-order), is the contraction sequence.
//
// Details the paper leaves open: the graph is the simple, unweighted tensor
// graph after rank <= 2 tensors are absorbed; betweenness is recomputed
// (Brandes' algorithm) inside the component that lost an edge; ties between
// edges go to the lowest edge index.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "graph.hpp"
#include "internal.hpp"

namespace tn {

namespace {

struct EdgeList {
    std::vector<std::pair<int32_t, int32_t>> ends;
    // live incidences only: vertex -> (neighbour, edge); a removed edge is
    // erased from both endpoints' lists, so no traversal tests for it
    std::vector<std::vector<std::pair<int32_t, int32_t>>> inc;
    std::vector<uint8_t> removed;
    void remove(int32_t e) {
        removed[size_t(e)] = 1;
        for (int32_t x : {ends[size_t(e)].first, ends[size_t(e)].second}) {
            auto& l = inc[size_t(x)];
            for (size_t k = 0; k < l.size(); ++k)
                if (l[k].second == e) {
                    l.erase(l.begin() + std::ptrdiff_t(k));
                    break;
                }
        }
    }
};

// Brandes edge betweenness restricted to the vertices of one component.
struct Brandes {
    std::vector<int32_t> dist, order;
    std::vector<double> sigma, delta;
    explicit Brandes(size_t n) : dist(n, -1), sigma(n, 0.0), delta(n, 0.0) { order.reserve(n); }
    void run(const EdgeList& el, const std::vector<int32_t>& comp, std::vector<double>& eb) {
        for (int32_t s : comp) {
            order.clear();
            for (int32_t v : comp) {
                dist[size_t(v)] = -1;
                sigma[size_t(v)] = 0.0;
                delta[size_t(v)] = 0.0;
            }
            dist[size_t(s)] = 0;
            sigma[size_t(s)] = 1.0;
            order.push_back(s);
            for (size_t h = 0; h < order.size(); ++h) {
                const int32_t v = order[h];
                const int32_t dv = dist[size_t(v)] + 1;
                const double sv = sigma[size_t(v)];
                for (const auto& pr : el.inc[size_t(v)]) {
                    const int32_t w = pr.first;
                    if (dist[size_t(w)] < 0) {
                        dist[size_t(w)] = dv;
                        order.push_back(w);
                    }
                    if (dist[size_t(w)] == dv) sigma[size_t(w)] += sv;
                }
            }
            for (size_t h = order.size(); h-- > 0;) {
                const int32_t w = order[h];
                const int32_t dw = dist[size_t(w)] - 1;
                const double sw = sigma[size_t(w)], dl = 1.0 + delta[size_t(w)];
                for (const auto& pr : el.inc[size_t(w)]) {
                    const int32_t v = pr.first;
                    if (dist[size_t(v)] == dw) {
                        const double c = sigma[size_t(v)] / sw * dl;
                        eb[size_t(pr.second)] += c;
                        delta[size_t(v)] += c;
                    }
                }
            }
        }
    }
};

std::vector<int32_t> reach(const EdgeList& el, int32_t s, std::vector<uint8_t>& seen) {
    std::vector<int32_t> out{s};
    seen[size_t(s)] = 1;
    for (size_t h = 0; h < out.size(); ++h)
        for (const auto& pr : el.inc[size_t(out[h])])
            if (!seen[size_t(pr.first)]) {
                seen[size_t(pr.first)] = 1;
                out.push_back(pr.first);
            }
    for (int32_t x : out) seen[size_t(x)] = 0;
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace

std::vector<std::pair<int32_t, int32_t>> order_community(const Network& net) {
    Reduced r = absorb_small(net);
    if (r.id.size() <= 1) return r.merges;
    WGraph g = reduced_graph(r, true);
    EdgeList el;
    el.inc.assign(g.n, {});
    for (int32_t v = 0; v < g.n; ++v)
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            if (v < g.adj[e]) {
                int32_t id = int32_t(el.ends.size());
                el.ends.push_back({v, g.adj[e]});
                el.inc[v].push_back({g.adj[e], id});
                el.inc[g.adj[e]].push_back({v, id});
            }
    el.removed.assign(el.ends.size(), 0);

    // a community is a sorted vertex list; communities that never split
    // are single vertices (the leaves)
    Tree tree;
    std::vector<int32_t> all(g.n);
    std::iota(all.begin(), all.end(), 0);
    auto comps = components(g, all);

    // the split tree is recorded as (parent community id -> two children);
    // communities are numbered as they appear
    std::vector<std::vector<int32_t>> comm_verts;
    std::vector<std::pair<int32_t, int32_t>> comm_kids;
    std::vector<int32_t> comm_of(g.n, -1);
    std::vector<int32_t> roots;
    for (const auto& c : comps) {
        int32_t id = int32_t(comm_verts.size());
        comm_verts.push_back(c);
        comm_kids.push_back({-1, -1});
        for (int32_t v : c) comm_of[v] = id;
        roots.push_back(id);
    }
    std::vector<double> eb(el.ends.size(), 0.0);
    std::vector<uint8_t> dirty(comm_verts.size(), 1);
    Brandes brandes(size_t(g.n));
    std::vector<uint8_t> seen(size_t(g.n), 0);
    // betweenness is kept per edge; recomputed for communities marked dirty
    int32_t live_edges = int32_t(el.ends.size());
    while (live_edges > 0) {
        for (int32_t cid = 0; cid < int32_t(comm_verts.size()); ++cid) {
            if (!dirty[cid] || comm_kids[cid].first >= 0) continue;
            for (int32_t v : comm_verts[cid])
                for (const auto& pr : el.inc[v])
                    if (v < pr.first) eb[pr.second] = 0.0;
            brandes.run(el, comm_verts[cid], eb);
            dirty[cid] = 0;
        }
        int32_t best = -1;
        for (int32_t e = 0; e < int32_t(el.ends.size()); ++e) {
            if (el.removed[e]) continue;
            if (best < 0 || eb[e] > eb[best] * (1.0 + 1e-12) + 1e-12) best = e;
        }
        el.remove(best);
        --live_edges;
        int32_t u = el.ends[best].first, v = el.ends[best].second;
        int32_t cid = comm_of[u];
        std::vector<int32_t> ru = reach(el, u, seen);
        if (std::binary_search(ru.begin(), ru.end(), v)) {
            dirty[cid] = 1;
            continue;
        }
        // the community split into the part holding u and the rest
        std::vector<int32_t> rv;
        std::set_difference(comm_verts[cid].begin(), comm_verts[cid].end(), ru.begin(), ru.end(),
                            std::back_inserter(rv));
        int32_t a = int32_t(comm_verts.size());
        comm_verts.push_back(ru);
        comm_kids.push_back({-1, -1});
        int32_t b = int32_t(comm_verts.size());
        comm_verts.push_back(rv);
        comm_kids.push_back({-1, -1});
        comm_kids[cid] = {a, b};
        for (int32_t x : ru) comm_of[x] = a;
        for (int32_t x : rv) comm_of[x] = b;
        dirty.push_back(1);
        dirty.push_back(1);
    }
    // communities with no split are single vertices (all edges removed)
    std::vector<int32_t> node_of(comm_verts.size(), 0);
    // children are numbered after parents, so a reverse sweep sees them first
    for (int32_t cid = int32_t(comm_verts.size()) - 1; cid >= 0; --cid) {
        if (comm_kids[cid].first < 0) {
            node_of[cid] = ~comm_verts[cid][0];
        } else {
            node_of[cid] = tree_node(tree, node_of[comm_kids[cid].first], node_of[comm_kids[cid].second]);
        }
    }
    int32_t root = node_of[roots[0]];
    for (size_t i = 1; i < roots.size(); ++i) root = tree_node(tree, root, node_of[roots[i]]);
    return merges_from_tree(r, tree, root);
}

}  // namespace tn
