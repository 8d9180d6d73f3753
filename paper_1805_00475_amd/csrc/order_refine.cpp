// Local refinement of a contraction tree.
//
// A plan's merges form a binary tree whose leaves are the original
// tensors. Any subtree, cut at some frontier of k nodes (leaves or deeper
// subtrees kept as they are), produces the same tensor whatever binary tree
// joins its k frontier nodes: the result's bonds are those of the frontier
// that leave the subtree. So the subtree's internal order can be replaced
// by the cheapest one, found exactly by dynamic programming over the 2^k
// subsets of the frontier (k <= 8), without changing the rest of the plan or
// the count. The cost of a merge is the plan's cost model; the frontier is
// grown from the subtree's root by opening the highest-rank internal node
// first. The first sweep visits every internal node, later ones only the
// nodes whose window a change can have reached, until none is left or the
// time budget is spent.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace tn {

namespace {

struct Tree {
    int32_t n_leaves = 0, words = 0;
    std::vector<int32_t> left, right, parent;  // per node id; leaves have -1 children
    std::vector<uint64_t> bonds;              // words per node
    int32_t root = -1;
    uint64_t* b(int32_t v) { return bonds.data() + size_t(v) * words; }
    int rank(int32_t v) const {
        int c = 0;
        for (int i = 0; i < words; ++i) c += __builtin_popcountll(bonds[size_t(v) * words + i]);
        return c;
    }
};

constexpr int kMaxFrontier = 8;
constexpr int kMaxSweeps = 6;

// set per refinement (per thread: orders are searched on worker threads):
// no intermediate may exceed the plan's largest rank; steps are priced in
// the network's default residue arithmetic
thread_local int g_rank_cap = 64;
thread_local int g_mode = RM_SMALL;

// step_cost_model by table for operands of rank below kTabRank (the DP
// evaluates it thousands of times per subtree), built once per mode
constexpr int kTabRank = 48;
const double* cost_table(int mode) {
    static std::once_flag once[3];
    static std::vector<double> tab[3];
    std::call_once(once[mode], [mode]() {
        std::vector<double>& t = tab[mode];
        t.assign(size_t(kTabRank) * kTabRank * kTabRank, 0.0);
        for (int ra = 0; ra < kTabRank; ++ra)
            for (int rb = 0; rb < kTabRank; ++rb)
                for (int s = 0; s <= std::min(ra, rb); ++s)
                    t[(size_t(ra) * kTabRank + rb) * kTabRank + s] = step_cost_model(ra, rb, s, ra + rb - 2 * s, mode);
    });
    return tab[mode].data();
}
thread_local const double* g_tab = nullptr;

double merge_cost(int ra, int rb, int rc) {
    const int s = (ra + rb - rc) / 2;
    const double c = ra < kTabRank && rb < kTabRank ? g_tab[(size_t(ra) * kTabRank + rb) * kTabRank + s]
                                                    : step_cost_model(ra, rb, s, rc, g_mode);
    return rc > g_rank_cap ? c + 1e15 : c;
}

double subtree_cost(Tree& t, int32_t v, const std::vector<char>& is_frontier) {
    if (is_frontier[v] || t.left[v] < 0) return 0.0;
    const int32_t a = t.left[v], c = t.right[v];
    return subtree_cost(t, a, is_frontier) + subtree_cost(t, c, is_frontier) +
           merge_cost(t.rank(a), t.rank(c), t.rank(v));
}

void collect_internal(Tree& t, int32_t v, const std::vector<char>& is_frontier, std::vector<int32_t>& out) {
    if (is_frontier[v] || t.left[v] < 0) return;
    out.push_back(v);
    collect_internal(t, t.left[v], is_frontier, out);
    collect_internal(t, t.right[v], is_frontier, out);
}

// Try to improve the subtree rooted at v; returns true when it changed,
// the ids of the internal nodes it rebuilt (v among them) in `rebuilt`.
bool reconfigure(Tree& t, int32_t v, std::vector<char>& is_frontier, std::vector<int32_t>& rebuilt) {
    if (t.left[v] < 0) return false;
    // grow the frontier from v's children, opening the highest-rank
    // internal node first
    // buffers kept per thread across calls (a refinement makes about a
    // thousand of them)
    thread_local std::vector<int32_t> fr, old_internal, pool;
    thread_local std::vector<uint64_t> sb;
    thread_local std::vector<int> sr, split;
    thread_local std::vector<double> cost;
    fr.assign({t.left[v], t.right[v]});
    while (int(fr.size()) < kMaxFrontier) {
        int best = -1, br = -1;
        for (int i = 0; i < int(fr.size()); ++i)
            if (t.left[fr[i]] >= 0 && t.rank(fr[i]) > br) {
                br = t.rank(fr[i]);
                best = i;
            }
        if (best < 0) break;
        const int32_t x = fr[size_t(best)];
        fr[size_t(best)] = t.left[x];
        fr.push_back(t.right[x]);
    }
    const int k = int(fr.size());
    if (k <= 2) return false;
    for (int32_t x : fr) is_frontier[x] = 1;
    const double old_cost = subtree_cost(t, v, is_frontier);
    old_internal.clear();
    collect_internal(t, v, is_frontier, old_internal);
    // DP over subsets of the frontier, on bond sets restricted to the bonds
    // the frontier nodes hold (every subset's result lies within them): at
    // most 8 x 64 bonds, so a few words instead of one bit per bond of the
    // network
    const int S = 1 << k;
    thread_local std::vector<int32_t> local_of;  // bond -> local index, -1 elsewhere
    thread_local std::vector<int32_t> held;
    thread_local std::vector<uint64_t> lbits;
    if (local_of.size() < size_t(t.words) * 64) local_of.assign(size_t(t.words) * 64, -1);
    held.clear();
    for (int32_t x : fr) {
        const uint64_t* bx = t.b(x);
        for (int w = 0; w < t.words; ++w)
            for (uint64_t word = bx[w]; word; word &= word - 1) {
                const int32_t bnd = w * 64 + __builtin_ctzll(word);
                if (local_of[size_t(bnd)] < 0) {
                    local_of[size_t(bnd)] = int32_t(held.size());
                    held.push_back(bnd);
                }
            }
    }
    const int W = int(held.size() + 63) / 64;
    lbits.assign(size_t(k) * W, 0);
    for (int i = 0; i < k; ++i) {
        const uint64_t* bx = t.b(fr[size_t(i)]);
        for (int w = 0; w < t.words; ++w)
            for (uint64_t word = bx[w]; word; word &= word - 1) {
                const int32_t l = local_of[size_t(w * 64 + __builtin_ctzll(word))];
                lbits[size_t(i) * W + size_t(l) / 64] |= uint64_t(1) << (l % 64);
            }
    }
    for (int32_t bnd : held) local_of[size_t(bnd)] = -1;
    sb.assign(size_t(S) * W, 0);
    sr.assign(size_t(S), 0);
    cost.assign(size_t(S), 0.0);
    split.assign(size_t(S), 0);
    for (int m = 1; m < S; ++m) {
        const int low = __builtin_ctz(m);
        const int rest = m & (m - 1);
        const uint64_t* lb = lbits.data() + size_t(low) * W;
        for (int i = 0; i < W; ++i) sb[size_t(m) * W + i] = sb[size_t(rest) * W + i] ^ lb[i];
        int c = 0;
        for (int i = 0; i < W; ++i) c += __builtin_popcountll(sb[size_t(m) * W + i]);
        sr[m] = c;
        if (rest == 0) continue;  // a single frontier node
        double best = 1e300;
        int bs = 0;
        // splits m = a | (m ^ a) with a containing the lowest element
        for (int a = (m - 1) & m; a > 0; a = (a - 1) & m) {
            if (!(a & (1 << low))) continue;
            const int bb = m ^ a;
            const double cst = cost[a] + cost[bb] + merge_cost(sr[a], sr[bb], c);
            if (cst < best) {
                best = cst;
                bs = a;
            }
        }
        cost[m] = best;
        split[m] = bs;
    }
    const int full = S - 1;
    bool changed = false;
    if (cost[full] < old_cost * (1.0 - 1e-9)) {
        // rebuild: reuse the k-1 internal node ids (v stays the root)
        pool.clear();
        for (int32_t x : old_internal)
            if (x != v) pool.push_back(x);
        // recursive assembly
        struct Builder {
            Tree& t;
            const std::vector<int32_t>& fr;
            const std::vector<int>& split;
            std::vector<int32_t>& pool;
            int32_t make(int m, int32_t id) {
                if ((m & (m - 1)) == 0) return fr[size_t(__builtin_ctz(m))];
                const int a = split[m], bb = m ^ a;
                const int32_t na = (a & (a - 1)) == 0 ? fr[size_t(__builtin_ctz(a))] : take();
                const int32_t nb = (bb & (bb - 1)) == 0 ? fr[size_t(__builtin_ctz(bb))] : take();
                if (na >= t.n_leaves && (a & (a - 1)) != 0) make(a, na);
                if (nb >= t.n_leaves && (bb & (bb - 1)) != 0) make(bb, nb);
                t.left[id] = na;
                t.right[id] = nb;
                t.parent[na] = id;
                t.parent[nb] = id;
                // the node's bonds: its children's, less the shared ones
                const uint64_t *ba = t.b(na), *bn = t.b(nb);
                uint64_t* bi = t.b(id);
                for (int w = 0; w < t.words; ++w) bi[w] = ba[w] ^ bn[w];
                return id;
            }
            int32_t take() {
                int32_t x = pool.back();
                pool.pop_back();
                return x;
            }
        } bld{t, fr, split, pool};
        bld.make(full, v);
        changed = true;
        rebuilt = old_internal;
    }
    for (int32_t x : fr) is_frontier[x] = 0;
    return changed;
}

}  // namespace

std::vector<std::pair<int32_t, int32_t>> refine_order(const Network& net,
                                                      const std::vector<std::pair<int32_t, int32_t>>& merges,
                                                      double budget_us) {
    const auto t0 = std::chrono::steady_clock::now();
    const int32_t n0 = int32_t(net.t.size());
    const int32_t n = n0 + int32_t(merges.size());
    if (merges.size() < 2) return merges;
    Tree t;
    t.n_leaves = n0;
    t.words = int32_t((net.bond_end.size() + 63) / 64) + 1;
    t.left.assign(n, -1);
    t.right.assign(n, -1);
    t.parent.assign(n, -1);
    t.bonds.assign(size_t(n) * t.words, 0);
    for (int32_t i = 0; i < n0; ++i)
        for (int32_t bnd : net.t[i].bonds) t.b(i)[bnd >> 6] ^= uint64_t(1) << (bnd & 63);
    for (int32_t k = 0; k < int32_t(merges.size()); ++k) {
        const int32_t v = n0 + k, a = merges[k].first, c = merges[k].second;
        t.left[v] = a;
        t.right[v] = c;
        t.parent[a] = t.parent[c] = v;
        for (int i = 0; i < t.words; ++i) t.b(v)[i] = t.b(a)[i] ^ t.b(c)[i];
    }
    t.root = n - 1;
    int maxr = 0;
    for (int32_t v = 0; v < n; ++v) maxr = std::max(maxr, t.rank(v));
    g_rank_cap = maxr;  // keep peak memory: never raise the largest rank
    g_mode = default_residue_mode(net.count_bits);
    g_tab = cost_table(g_mode);
    std::vector<char> is_frontier(n, 0);
    // Sweeps over the internal nodes still marked, largest tensors first
    // (their subtrees dominate the cost). A node is marked at the start and
    // again when a change can reach its window: the window of a node holds
    // nodes at most kMaxFrontier - 1 levels below it, and the bonds of a
    // node depend only on its leaves, so a rebuild at v can only change the
    // windows of the nodes it rebuilt and of v's ancestors within those
    // levels. Once nothing is marked, no window can improve.
    std::vector<char> marked(n, 0);
    for (int32_t v = n0; v < n; ++v) marked[v] = 1;
    std::vector<int32_t> rebuilt;
    bool stop = false;
    for (int sweep = 0; sweep < kMaxSweeps && !stop; ++sweep) {
        std::vector<int32_t> nodes;
        for (int32_t v = n0; v < n; ++v)
            if (marked[v]) nodes.push_back(v);
        if (nodes.empty()) break;
        std::sort(nodes.begin(), nodes.end(), [&](int32_t x, int32_t y) { return t.rank(x) > t.rank(y); });
        for (int32_t v : nodes) {
            if (!marked[v]) continue;
            marked[v] = 0;
            if (reconfigure(t, v, is_frontier, rebuilt)) {
                for (int32_t x : rebuilt) marked[x] = 1;
                int32_t a = t.parent[v];
                for (int d = 0; d < kMaxFrontier - 1 && a >= 0; ++d, a = t.parent[a]) marked[a] = 1;
            }
            const double spent =
                std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
            if (spent > budget_us) {
                stop = true;
                break;
            }
        }
    }
    // post-order from the root; new merge ids are assigned in that order
    std::vector<std::pair<int32_t, int32_t>> out;
    out.reserve(merges.size());
    std::vector<int32_t> newid(n, -1);
    for (int32_t i = 0; i < n0; ++i) newid[i] = i;
    int32_t next = n0;
    std::vector<std::pair<int32_t, int>> st = {{t.root, 0}};
    while (!st.empty()) {
        auto& top = st.back();
        const int32_t v = top.first;
        if (v < n0) {
            st.pop_back();
            continue;
        }
        if (top.second == 0) {
            top.second = 1;
            st.push_back({t.right[v], 0});
            st.push_back({t.left[v], 0});
            continue;
        }
        st.pop_back();
        const int32_t a = newid[t.left[v]], c = newid[t.right[v]];
        out.push_back({std::min(a, c), std::max(a, c)});
        newid[v] = next++;
    }
    return out;
}

}  // namespace tn
