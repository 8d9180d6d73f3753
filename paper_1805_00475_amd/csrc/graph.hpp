// Host graph helpers for the ordering heuristics.
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace tn {

// Live tensors of a network under a sequence of pairwise merges. Ids of
// merged tensors continue after the initial ones. For every live tensor:
// its rank, its sorted bond set and its neighbours with the number of bonds
// shared with each.
struct LiveGraph {
    std::vector<char> alive;
    std::vector<int32_t> rank;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> nb;
    std::vector<std::vector<int32_t>> bonds;
    int32_t next_id = 0;
    int32_t n_alive = 0;

    void init(const Network& net);
    void add_count(int32_t u, int32_t v, int32_t c);
    int32_t shared(int32_t u, int32_t v) const;
    int32_t merge(int32_t a, int32_t b);  // returns the new id
    void close_scalars(std::vector<std::pair<int32_t, int32_t>>& merges);
};

// Undirected weighted graph in compressed adjacency form.
struct WGraph {
    int32_t n = 0;
    std::vector<int32_t> xadj;  // n + 1
    std::vector<int32_t> adj;
    std::vector<int32_t> ew;    // edge weights, parallel to adj
    std::vector<int32_t> vw;    // vertex weights
    int64_t total_vw() const {
        int64_t s = 0;
        for (int32_t w : vw) s += w;
        return s;
    }
};

// Small deterministic PRNG (SplitMix64) for the randomized bisections.
struct SplitMix {
    uint64_t s;
    explicit SplitMix(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint32_t below(uint32_t n) { return uint32_t(next() % n); }
};

// Balanced min-cut bisection (multilevel: heavy-edge coarsening, every
// split of a coarsest graph of at most 12 vertices or else greedy graph
// growing, Fiduccia-Mattheyses refinement). Returns side 0/1 per vertex and
// the cut weight; *deterministic (if given) tells whether the result used
// no random draw (every split of the graph itself was tried).
std::vector<uint8_t> bisect(const WGraph& g, SplitMix& rng, int64_t* cut, bool* deterministic = nullptr);

// A binary contraction tree over vertex indices 0..n-1 of some graph:
// children of internal node k are kids[k]; leaves are encoded as ~vertex.
struct Tree {
    std::vector<std::pair<int32_t, int32_t>> kids;
    int32_t root = 0;
};

// Builds tree nodes: a leaf for vertex v is ~v; node(l, r) appends an
// internal node and returns its index.
inline int32_t tree_node(Tree& t, int32_t l, int32_t r) {
    t.kids.push_back({l, r});
    return int32_t(t.kids.size()) - 1;
}

// Absorption merges followed by the post-order merges of a tree over the
// reduced vertices (leaf v stands for tensor r.id[v]).
std::vector<std::pair<int32_t, int32_t>> merges_from_tree(const Reduced& r, const Tree& t, int32_t root);

// The partition order's input, the same for every trial of an order
// search: the network with its tensors of rank <= 2 absorbed, as a
// weighted graph.
struct PartitionInput {
    Reduced r;
    WGraph g;
};
PartitionInput partition_input(const Network& net);
std::vector<std::pair<int32_t, int32_t>> order_partition(const PartitionInput& in, uint64_t seed);

WGraph reduced_graph(const Reduced& r, bool unit_weights);
std::vector<std::vector<int32_t>> components(const WGraph& g, const std::vector<int32_t>& verts);

}  // namespace tn
