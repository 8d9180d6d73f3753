// tensor-METIS style order (Sec. 3.1.1): recursively bisect the tensor graph
// into two parts of roughly equal size cutting as few bonds as possible,
// computing every bisection twice from different random starts and keeping
// the better one, down to single tensors; the resulting separator hierarchy
// is contracted bottom-up, the smallest separators first (Corollary 1 and
// Fig. 2): post-order, each subtree reduced to one tensor before its parent
// merge.
//
// The bisection is this library's own multilevel scheme in the spirit of
// METIS: heavy-edge matching to coarsen, for the initial cut every split of
// the coarsest graph when it has at most 12 vertices, else greedy graph
// growing from random vertices, Fiduccia-Mattheyses refinement while
// uncoarsening. Before partitioning, tensors of rank <= 2 are absorbed into
// a neighbour (this never raises a rank); vertex weight 1 per remaining
// tensor, edge weight = number of bonds shared.
#include <algorithm>
#include <numeric>

#include "graph.hpp"
#include "internal.hpp"

namespace tn {

WGraph reduced_graph(const Reduced& r, bool unit_weights) {
    // bond -> owning reduced vertices
    int32_t maxb = -1;
    for (const auto& b : r.bonds)
        for (int32_t x : b) maxb = std::max(maxb, x);
    std::vector<int32_t> o1(size_t(maxb + 1), -1), o2(size_t(maxb + 1), -1);
    for (int32_t v = 0; v < int32_t(r.bonds.size()); ++v)
        for (int32_t x : r.bonds[v]) (o1[x] < 0 ? o1[x] : o2[x]) = v;
    const int32_t n = int32_t(r.bonds.size());
    std::vector<std::vector<std::pair<int32_t, int32_t>>> al(n);
    auto bump = [&](int32_t u, int32_t v) {
        for (auto& pr : al[u])
            if (pr.first == v) {
                pr.second += 1;
                return;
            }
        al[u].push_back({v, 1});
    };
    for (int32_t x = 0; x <= maxb; ++x)
        if (o1[x] >= 0 && o2[x] >= 0 && o1[x] != o2[x]) {
            bump(o1[x], o2[x]);
            bump(o2[x], o1[x]);
        }
    WGraph g;
    g.n = n;
    g.xadj.assign(n + 1, 0);
    g.vw.assign(n, 1);
    for (int32_t v = 0; v < n; ++v) {
        std::sort(al[v].begin(), al[v].end());
        for (const auto& pr : al[v]) {
            g.adj.push_back(pr.first);
            g.ew.push_back(unit_weights ? 1 : pr.second);
        }
        g.xadj[v + 1] = int32_t(g.adj.size());
    }
    return g;
}

// Connected components of the subgraph induced by verts; mark has g.n
// entries, -2 on entry and again on return (only verts' entries are touched).
std::vector<std::vector<int32_t>> components(const WGraph& g, const std::vector<int32_t>& verts,
                                             std::vector<int32_t>& mark) {
    for (int32_t v : verts) mark[v] = -1;
    std::vector<std::vector<int32_t>> comps;
    for (int32_t v : verts) {
        if (mark[v] != -1) continue;
        std::vector<int32_t> comp{v};
        mark[v] = int32_t(comps.size());
        for (size_t h = 0; h < comp.size(); ++h) {
            int32_t u = comp[h];
            for (int32_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
                int32_t w = g.adj[e];
                if (mark[w] == -1) {
                    mark[w] = int32_t(comps.size());
                    comp.push_back(w);
                }
            }
        }
        std::sort(comp.begin(), comp.end());
        comps.push_back(std::move(comp));
    }
    for (int32_t v : verts) mark[v] = -2;
    return comps;
}

std::vector<std::vector<int32_t>> components(const WGraph& g, const std::vector<int32_t>& verts) {
    std::vector<int32_t> mark(g.n, -2);
    return components(g, verts, mark);
}

namespace {

// the subgraph induced by verts, vertex i being verts[i]; local has g.n
// entries, -1 on entry and again on return
WGraph induced(const WGraph& g, const std::vector<int32_t>& verts, std::vector<int32_t>& local) {
    for (int32_t i = 0; i < int32_t(verts.size()); ++i) local[verts[i]] = i;
    WGraph h;
    h.n = int32_t(verts.size());
    h.xadj.assign(h.n + 1, 0);
    for (int32_t i = 0; i < h.n; ++i) {
        int32_t v = verts[i];
        h.vw.push_back(g.vw[v]);
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            if (local[g.adj[e]] >= 0) {
                h.adj.push_back(local[g.adj[e]]);
                h.ew.push_back(g.ew[e]);
            }
        h.xadj[i + 1] = int32_t(h.adj.size());
    }
    for (int32_t v : verts) local[v] = -1;
    return h;
}

int64_t cut_of(const WGraph& g, const std::vector<uint8_t>& side) {
    int64_t c = 0;
    for (int32_t v = 0; v < g.n; ++v)
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            if (side[v] != side[g.adj[e]]) c += g.ew[e];
    return c / 2;
}

struct Balance {
    int64_t lo, hi;  // allowed weight of side 0
};

Balance balance_of(const WGraph& g) {
    int64_t W = g.total_vw();
    int64_t maxw = 0;
    for (int32_t w : g.vw) maxw = std::max<int64_t>(maxw, w);
    int64_t tol = std::max<int64_t>(maxw, (W * 5 + 99) / 100);
    int64_t lo = std::max<int64_t>(1, W / 2 - tol);
    int64_t hi = std::min<int64_t>(W - 1, (W + 1) / 2 + tol);
    if (lo > hi) lo = hi = W / 2;
    return {lo, hi};
}

// Fiduccia-Mattheyses passes: move the unlocked vertex of best gain that
// keeps the balance, remember the best prefix of moves, undo the rest.
void fm_refine(const WGraph& g, std::vector<uint8_t>& side, int max_passes) {
    const Balance bal = balance_of(g);
    int64_t w0 = 0;
    for (int32_t v = 0; v < g.n; ++v)
        if (side[v] == 0) w0 += g.vw[v];
    const int64_t W = g.total_vw();
    // buffers kept per thread across calls (a trial refines hundreds of
    // small graphs)
    thread_local std::vector<int64_t> gain;
    thread_local std::vector<uint8_t> locked;
    thread_local std::vector<int32_t> moves;
    thread_local std::vector<std::pair<int64_t, int32_t>> heap[2];
    gain.assign(size_t(g.n), 0);
    locked.assign(size_t(g.n), 0);
    bool unit = true;
    for (int32_t v = 0; v < g.n; ++v) unit = unit && g.vw[v] == 1;
    for (int pass = 0; pass < max_passes; ++pass) {
        for (int32_t v = 0; v < g.n; ++v) {
            int64_t gv = 0;
            for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) gv += side[g.adj[e]] != side[v] ? g.ew[e] : -g.ew[e];
            gain[v] = gv;
        }
        std::fill(locked.begin(), locked.end(), 0);
        moves.clear();
        int64_t cur = 0, best = 0;
        size_t best_k = 0;
        int64_t best_dev = std::llabs(2 * w0 - W);
        int64_t cw0 = w0;
        // with unit vertex weights every vertex of a side is allowed or not
        // alike, so the best candidate is the top of one of two heaps
        // (largest gain, then lowest index; stale entries skipped): binary
        // max-heaps over (gain, -index)
        auto push = [&](int sd, int64_t gv, int32_t v) {
            heap[sd].push_back({gv, -v});
            std::push_heap(heap[sd].begin(), heap[sd].end());
        };
        heap[0].clear();
        heap[1].clear();
        if (unit)
            for (int32_t v = 0; v < g.n; ++v) push(side[v], gain[v], v);
        auto allowed = [&](int64_t wv, int from) {
            const int64_t nw0 = from == 0 ? cw0 - wv : cw0 + wv;
            // a move out of an unbalanced state toward balance is allowed
            return (nw0 >= bal.lo && nw0 <= bal.hi) || std::llabs(2 * nw0 - W) < std::llabs(2 * cw0 - W);
        };
        for (int32_t it = 0; it < g.n; ++it) {
            int32_t pick = -1;
            if (unit) {
                for (int sd = 0; sd < 2; ++sd) {
                    auto& h = heap[sd];
                    while (!h.empty()) {
                        const int32_t v = -h.front().second;
                        if (locked[v] || side[v] != sd || h.front().first != gain[v]) {
                            std::pop_heap(h.begin(), h.end());
                            h.pop_back();
                        } else {
                            break;
                        }
                    }
                    if (h.empty() || !allowed(1, sd)) continue;
                    const int32_t v = -h.front().second;
                    if (pick < 0 || gain[v] > gain[pick] || (gain[v] == gain[pick] && v < pick)) pick = v;
                }
            } else {
                for (int32_t v = 0; v < g.n; ++v) {
                    if (locked[v] || !allowed(g.vw[v], side[v])) continue;
                    if (pick < 0 || gain[v] > gain[pick]) pick = v;
                }
            }
            if (pick < 0) break;
            cur -= gain[pick];
            cw0 = side[pick] == 0 ? cw0 - g.vw[pick] : cw0 + g.vw[pick];
            side[pick] ^= 1;
            locked[pick] = 1;
            moves.push_back(pick);
            gain[pick] = -gain[pick];
            for (int32_t e = g.xadj[pick]; e < g.xadj[pick + 1]; ++e) {
                int32_t u = g.adj[e];
                // edge (pick,u) changed from cut to uncut or back
                gain[u] += side[u] == side[pick] ? -2 * g.ew[e] : 2 * g.ew[e];
                if (unit && !locked[u]) push(side[u], gain[u], u);
            }
            int64_t dev = std::llabs(2 * cw0 - W);
            bool inb = cw0 >= bal.lo && cw0 <= bal.hi;
            if (inb && (cur < best || (cur == best && dev < best_dev))) {
                best = cur;
                best_k = moves.size();
                best_dev = dev;
            }
        }
        for (size_t k = moves.size(); k > best_k; --k) {
            int32_t v = moves[k - 1];
            side[v] ^= 1;
        }
        w0 = 0;
        for (int32_t v = 0; v < g.n; ++v)
            if (side[v] == 0) w0 += g.vw[v];
        if (best_k == 0) break;
    }
}

// Greedy graph growing: start side 0 at a random vertex, repeatedly add
// the boundary vertex whose move lowers the cut most, until side 0 holds
// half the weight.
std::vector<uint8_t> grow(const WGraph& g, SplitMix& rng) {
    std::vector<uint8_t> side(g.n, 1);
    const int64_t W = g.total_vw();
    int32_t seed = int32_t(rng.below(uint32_t(g.n)));
    // gain of moving each side-1 vertex to side 0 (edges to side 0 minus
    // edges to side 1) and whether it touches side 0, kept up to date as
    // vertices move
    std::vector<int64_t> gv(g.n, 0);
    std::vector<uint8_t> boundary(g.n, 0);
    for (int32_t v = 0; v < g.n; ++v)
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) gv[v] -= g.ew[e];
    auto move = [&](int32_t p) {
        side[p] = 0;
        for (int32_t e = g.xadj[p]; e < g.xadj[p + 1]; ++e) {
            gv[g.adj[e]] += 2 * g.ew[e];
            boundary[g.adj[e]] = 1;
        }
    };
    move(seed);
    int64_t w0 = g.vw[seed];
    while (2 * w0 < W) {
        int32_t pick = -1;
        int64_t pg = 0;
        for (int32_t v = 0; v < g.n; ++v) {
            if (side[v] == 0) continue;
            const int64_t key = boundary[v] ? gv[v] : gv[v] - (1 << 20);  // prefer staying connected
            if (pick < 0 || key > pg) {
                pick = v;
                pg = key;
            }
        }
        if (pick < 0) break;
        move(pick);
        w0 += g.vw[pick];
    }
    return side;
}

// graphs up to this many vertices are bisected by trying every split
constexpr int32_t kExactBisect = 12;

// Exhaustive balanced bisection of a small graph: vertex 0 stays on side 0
// (the sides are interchangeable and the balance window is symmetric) and
// the other vertices run through every split in Gray-code order, one vertex
// changing side per step so that the cut and the weight update in O(degree).
// The lightest cut within the window wins, then the split closer to even,
// then the earlier one. Empty when no split is within the window.
std::vector<uint8_t> exact_bisect(const WGraph& g) {
    const Balance bal = balance_of(g);
    const int64_t W = g.total_vw();
    std::vector<uint8_t> side(g.n, 0), best;
    int64_t w0 = W, c = 0, bestc = -1, bestdev = 0;
    for (uint32_t i = 0; i < (uint32_t(1) << (g.n - 1)); ++i) {
        if (i > 0) {
            const int32_t v = 1 + __builtin_ctz(i);
            for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) c += side[g.adj[e]] == side[v] ? g.ew[e] : -g.ew[e];
            w0 += side[v] == 0 ? -g.vw[v] : g.vw[v];
            side[v] ^= 1;
        }
        if (w0 < bal.lo || w0 > bal.hi) continue;
        const int64_t dev = std::llabs(2 * w0 - W);
        if (bestc < 0 || c < bestc || (c == bestc && dev < bestdev)) {
            bestc = c;
            bestdev = dev;
            best = side;
        }
    }
    return best;
}

// One level of heavy-edge matching; cmap maps fine -> coarse vertex.
WGraph coarsen(const WGraph& g, SplitMix& rng, std::vector<int32_t>& cmap) {
    std::vector<int32_t> perm(g.n);
    std::iota(perm.begin(), perm.end(), 0);
    for (int32_t i = g.n - 1; i > 0; --i) std::swap(perm[i], perm[rng.below(uint32_t(i + 1))]);
    std::vector<int32_t> match(g.n, -1);
    for (int32_t v : perm) {
        if (match[v] >= 0) continue;
        int32_t best = -1, bw = -1;
        for (int32_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            int32_t u = g.adj[e];
            if (match[u] < 0 && u != v && g.ew[e] > bw) {
                best = u;
                bw = g.ew[e];
            }
        }
        if (best >= 0) {
            match[v] = best;
            match[best] = v;
        } else {
            match[v] = v;
        }
    }
    cmap.assign(g.n, -1);
    int32_t nc = 0;
    for (int32_t v = 0; v < g.n; ++v)
        if (cmap[v] < 0) {
            cmap[v] = nc;
            cmap[match[v]] = nc;
            ++nc;
        }
    // coarse adjacency, one coarse vertex at a time (its one or two fine
    // members in index order): neighbours and summed weights gathered through
    // a position table, then sorted by neighbour
    WGraph c;
    c.n = nc;
    c.vw.assign(nc, 0);
    c.xadj.assign(nc + 1, 0);
    c.adj.reserve(g.adj.size());
    c.ew.reserve(g.adj.size());
    std::vector<int32_t> pos(nc, -1);
    std::vector<std::pair<int32_t, int32_t>> row;
    int32_t a = 0;
    for (int32_t v = 0; v < g.n; ++v) {
        if (cmap[v] != a) continue;  // v is not the first member of a new coarse vertex
        const int32_t members[2] = {v, match[v]};
        const int nm = match[v] == v ? 1 : 2;
        row.clear();
        for (int k = 0; k < nm; ++k) {
            const int32_t u = members[k];
            c.vw[a] += g.vw[u];
            for (int32_t e = g.xadj[u]; e < g.xadj[u + 1]; ++e) {
                const int32_t b = cmap[g.adj[e]];
                if (b == a) continue;
                if (pos[b] < 0) {
                    pos[b] = int32_t(row.size());
                    row.push_back({b, g.ew[e]});
                } else {
                    row[size_t(pos[b])].second += g.ew[e];
                }
            }
        }
        std::sort(row.begin(), row.end());
        for (const auto& pr : row) {
            c.adj.push_back(pr.first);
            c.ew.push_back(pr.second);
            pos[pr.first] = -1;
        }
        c.xadj[a + 1] = int32_t(c.adj.size());
        ++a;
    }
    return c;
}

}  // namespace

std::vector<uint8_t> bisect(const WGraph& g, SplitMix& rng, int64_t* cut, bool* deterministic) {
    if (deterministic) *deterministic = false;
    if (g.n <= 1) {
        if (cut) *cut = 0;
        if (deterministic) *deterministic = true;
        return std::vector<uint8_t>(g.n, 0);
    }
    std::vector<WGraph> levels{g};
    std::vector<std::vector<int32_t>> maps;
    while (levels.back().n > 24) {
        std::vector<int32_t> cm;
        WGraph c = coarsen(levels.back(), rng, cm);
        if (c.n > levels.back().n * 9 / 10) break;
        maps.push_back(std::move(cm));
        levels.push_back(std::move(c));
    }
    const WGraph& top = levels.back();
    std::vector<uint8_t> best;
    int64_t bestcut = -1;
    if (top.n <= kExactBisect) best = exact_bisect(top);
    // every split of the graph itself tried, no random draw made
    if (deterministic) *deterministic = !best.empty() && maps.empty();
    const int grow_trials = best.empty() ? 6 : 0;
    for (int t = 0; t < grow_trials; ++t) {
        std::vector<uint8_t> side = grow(top, rng);
        fm_refine(top, side, 8);
        int64_t c = cut_of(top, side);
        if (bestcut < 0 || c < bestcut) {
            bestcut = c;
            best = side;
        }
    }
    std::vector<uint8_t> side = best;
    for (int32_t L = int32_t(maps.size()) - 1; L >= 0; --L) {
        const WGraph& fine = levels[L];
        std::vector<uint8_t> fs(fine.n);
        for (int32_t v = 0; v < fine.n; ++v) fs[v] = side[maps[L][v]];
        fm_refine(fine, fs, 8);
        side = std::move(fs);
    }
    // never return an empty side
    int32_t n0 = 0;
    for (uint8_t s : side) n0 += s == 0;
    if (n0 == 0 || n0 == g.n) {
        for (int32_t v = 0; v < g.n; ++v) side[v] = v < g.n / 2 ? 0 : 1;
    }
    if (cut) *cut = cut_of(g, side);
    return side;
}

std::vector<std::pair<int32_t, int32_t>> merges_from_tree(const Reduced& r, const Tree& t, int32_t root) {
    std::vector<std::pair<int32_t, int32_t>> merges = r.merges;
    int32_t next = r.next_id;
    // iterative post-order
    std::vector<std::pair<int32_t, int>> st;  // (node, state)
    std::vector<int32_t> val;                // tensor id of finished subtrees
    if (r.id.empty()) return merges;
    st.push_back({root, 0});
    while (!st.empty()) {
        auto& top = st.back();
        int32_t node = top.first;
        if (node < 0) {
            val.push_back(r.id[~node]);
            st.pop_back();
            continue;
        }
        if (top.second == 0) {
            top.second = 1;
            st.push_back({t.kids[node].second, 0});
            st.push_back({t.kids[node].first, 0});
            continue;
        }
        st.pop_back();
        int32_t b = val.back();
        val.pop_back();
        int32_t a = val.back();
        val.pop_back();
        merges.push_back({std::min(a, b), std::max(a, b)});
        val.push_back(next++);
    }
    return merges;
}

namespace {

struct PartitionBuilder {
    const WGraph& g;
    SplitMix rng;
    Tree tree;
    std::vector<int32_t> mark, local;  // scratch over g's vertices (components, induced)
    PartitionBuilder(const WGraph& g_, uint64_t seed) : g(g_), rng(seed), mark(g_.n, -2), local(g_.n, -1) {}

    // join subtrees left to right (outer products of independent parts)
    int32_t chain(const std::vector<int32_t>& nodes) {
        int32_t acc = nodes[0];
        for (size_t i = 1; i < nodes.size(); ++i) acc = tree_node(tree, acc, nodes[i]);
        return acc;
    }

    int32_t build(const std::vector<int32_t>& verts) {
        if (verts.size() == 1) return ~verts[0];
        auto comps = components(g, verts, mark);
        if (comps.size() > 1) {
            std::sort(comps.begin(), comps.end(),
                      [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
                          return a.size() != b.size() ? a.size() < b.size() : a[0] < b[0];
                      });
            std::vector<int32_t> nodes;
            for (const auto& c : comps) nodes.push_back(build(c));
            return chain(nodes);
        }
        WGraph h = induced(g, verts, local);
        // best of two bisections (Sec. 3.1.1); when the first tried every
        // split without a random draw, the second would repeat it
        int64_t c1 = 0, c2 = 0;
        bool same = false;
        std::vector<uint8_t> s1 = bisect(h, rng, &c1, &same);
        std::vector<uint8_t> s2 = same ? std::vector<uint8_t>() : bisect(h, rng, &c2);
        const std::vector<uint8_t>& s = !same && c2 < c1 ? s2 : s1;
        std::vector<int32_t> L, R;
        for (int32_t i = 0; i < h.n; ++i) (s[i] == 0 ? L : R).push_back(verts[i]);
        return tree_node(tree, build(L), build(R));
    }
};

}  // namespace

PartitionInput partition_input(const Network& net) {
    PartitionInput in;
    in.r = absorb_small(net);
    if (in.r.id.size() > 1) in.g = reduced_graph(in.r, false);
    return in;
}

std::vector<std::pair<int32_t, int32_t>> order_partition(const PartitionInput& in, uint64_t seed) {
    if (in.r.id.size() <= 1) return in.r.merges;
    PartitionBuilder pb(in.g, seed ^ 0x5EEDB15EC7ull);
    std::vector<int32_t> all(in.g.n);
    std::iota(all.begin(), all.end(), 0);
    int32_t root = pb.build(all);
    return merges_from_tree(in.r, pb.tree, root);
}

std::vector<std::pair<int32_t, int32_t>> order_partition(const Network& net, uint64_t seed) {
    return order_partition(partition_input(net), seed);
}

}  // namespace tn
