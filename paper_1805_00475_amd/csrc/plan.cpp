// Plan: from a list of pairwise merges to everything the GPU loop needs --
// the bit order of every tensor, the per-step kernel parameters, the arena
// offsets, and the predicted cost (the "lazy" evaluation of Sec. 4: contract
// the graph first, track ranks, and know the cost before any entry is
// touched).
//
// Layout convention. Every bond dies at exactly one step (the step where
// the two tensors holding it merge). Each tensor lists its bonds sorted by
// death step, earliest first (bond id on ties); bit 0 of an entry's index
// is the earliest-dying bond. The bonds shared by the two operands of a step
// die at that step and every other bond of either operand dies later, so
// the shared bonds are the low s bits of both operands, in the same order:
// A = [z | xA] and B = [z | xB], and C's bits are the free bonds of A and B
// merged in death order -- which is again the layout C's own consumer needs.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>

#include "internal.hpp"

namespace tn {

namespace {

int64_t align_up(int64_t x) { return (x + kAlignElems - 1) / kAlignElems * kAlignElems; }

// First-fit arena over [0, inf) with coalescing free list.
struct Arena {
    std::map<int64_t, int64_t> free_;  // offset -> size
    int64_t top = 0;
    int64_t high = 0;
    int64_t alloc(int64_t n) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                int64_t off = it->first;
                int64_t rest = it->second - n;
                free_.erase(it);
                if (rest > 0) free_[off + n] = rest;
                return off;
            }
        // extend: reuse a free block touching the top
        int64_t off = top;
        if (!free_.empty()) {
            auto last = std::prev(free_.end());
            if (last->first + last->second == top) {
                off = last->first;
                free_.erase(last);
            }
        }
        top = off + n;
        high = std::max(high, top);
        return off;
    }
    void release(int64_t off, int64_t n) {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        if (it->first + it->second == top) {
            top = it->first;
            free_.erase(it);
        }
    }
};

}  // namespace

int default_residue_mode(int32_t count_bits) {
    if (count_bits <= 63) return RM_U64;
    return small_moduli_needed(count_bits) > 0 ? RM_SMALL : RM_WIDE;
}

int32_t default_planes(int32_t count_bits) {
    switch (default_residue_mode(count_bits)) {
        case RM_U64: return 1;
        case RM_SMALL: return small_moduli_needed(count_bits);
        default: return primes_needed(count_bits);
    }
}

// Predicted device time in microseconds of one step for one residue plane,
// launch excluded, from the kernels' measured behaviour on MI355X
// (single-instance contractions of cubic vertex-cover and 1-in-3 formulas,
// n = 80..225, fitted per kernel class).
//  - small moduli (1-byte entries): the int8 matrix-core kernels (larger free
//    side >= 7 bits, smaller >= 6, any K) take 1 / 1.5e15 s per multiply-add
//    plus the entries read and written at 2e12 B/s (within 15 % from K = 2^5
//    to 2^13: small K is bound by the output write, large K by the matrix
//    cores at about 60 % of the int8 peak); the split-K dot (rC <= 6,
//    s >= 10) moves its bytes at 1.8e12 B/s, the narrow matrix-core kernel
//    (B side of at most 64 rows, s >= 6; A read once) at NARROW_BPS plus the
//    int8 rate, streaming steps (s <= 5) at 7e11 B/s.
//  - 64-bit counts and 16-bit primes: the wave-per-output kernel (s >= 6,
//    narrow sides) at 4e10 B/s.
//  - 64-bit counts (8-byte entries, no matrix cores): the same non-matrix
//    classes.
//  - 16-bit primes (4-byte entries): the int8-limb matrix-core kernel at the
//    int8 peak (8 ops per modular multiply-add: four digit-pair products)
//    times an efficiency that grows with K (the per-tile epilogue is
//    amortized; table for s = 6..13 and beyond) plus a digit pass over both
//    operands (4 bytes read, 2 written per entry) and the output write;
//    other steps as above with 4-byte entries.
double step_cost_model(int rA, int rB, int s, int rC, int mode) {
    const double ea = std::ldexp(1.0, rA), eb = std::ldexp(1.0, rB), ec = std::ldexp(1.0, rC);
    const double macs = std::ldexp(1.0, rA + rB - s);
    const int fa = std::max(rA, rB) - s, fb = std::min(rA, rB) - s;
    const double es = mode == RM_U64 ? 8.0 : mode == RM_WIDE ? 4.0 : 1.0;
    const double bytes = es * (ea + eb + ec);
    double t;
    constexpr double NARROW_BPS = 3e12;
    if (mode == RM_SMALL && fa >= 7 && fb >= 6) {
        t = macs / 1.5e15 + bytes / 2e12;
    } else if (mode == RM_SMALL && s >= 6 && !(s >= 10 && rC <= 6) && (fb <= 5 || (fb == 6 && fa < 7))) {
        t = macs / 1.5e15 + bytes / NARROW_BPS;
    } else if (mode == RM_WIDE && s >= 6 && fa >= 7 && fb >= 6) {
        static const double eff[] = {0.042, 0.087, 0.12, 0.22, 0.31, 0.39, 0.45, 0.45};
        const double e = eff[std::min(s, 13) - 6];
        t = macs * 8.0 / (5e15 * e) + 6.0 * (ea + eb) / 5e12 + 4.0 * ec / 2.5e12;
    } else if (s >= 10 && rC <= 6) {
        t = bytes / 1.8e12;  // split-K dot
    } else if (s >= 6) {
        t = bytes / 4e10;
    } else {
        t = bytes / 7e11;
    }
    return 1e6 * t;
}

namespace {

// A plan's predicted device time, accumulated one step at a time in plan
// order (every residue plane, launches included); make_plan and
// sketch_plan both sum through it, so that a sketch's cost is the full
// plan's to the last bit.
struct CostSum {
    static constexpr int kPlanesPerLaunch = 16;  // residue planes of one launch
    static constexpr double kLaunchUs = 5.0;
    int mode;
    int32_t planes;
    double launches;
    double t = 0;
    explicit CostSum(int32_t count_bits)
        : mode(default_residue_mode(count_bits)),
          planes(default_planes(count_bits)),
          launches(double((planes + kPlanesPerLaunch - 1) / kPlanesPerLaunch)) {}
    void add(int rA, int rB, int s, int rC) { t += planes * step_cost_model(rA, rB, s, rC, mode) + launches * kLaunchUs; }
};

}  // namespace

double plan_cost(const Plan& plan) {
    if (plan.cost_us >= 0) return plan.cost_us;
    CostSum c(plan.count_bits);
    for (const Step& st : plan.steps) c.add(st.rA, st.rB, st.s, st.rC);
    return c.t;
}

tn_status sketch_plan(const Network& net, std::vector<std::pair<int32_t, int32_t>> merges, int32_t chosen,
                      Plan& plan) {
    try {
        const int32_t n_init = int32_t(net.t.size());
        const int32_t n_ids = n_init + int32_t(merges.size());
        const int32_t W = int32_t((net.bond_end.size() + 63) / 64) + 1;
        // bond sets as bit sets: C's bonds are A's and B's less the shared ones
        std::vector<uint64_t> bits(size_t(n_ids) * size_t(W), 0);
        std::vector<int32_t> rank(size_t(n_ids), 0);
        std::vector<int8_t> state(size_t(n_ids), 0);  // 0 unborn, 1 live, 2 consumed
        int32_t maxr = 0;
        for (int32_t i = 0; i < n_init; ++i) {
            uint64_t* b = bits.data() + size_t(i) * W;
            for (int32_t bnd : net.t[i].bonds) {
                if ((b[bnd >> 6] >> (bnd & 63)) & 1) return TN_EINVAL;
                b[bnd >> 6] |= uint64_t(1) << (bnd & 63);
            }
            rank[i] = int32_t(net.t[i].bonds.size());
            maxr = std::max(maxr, rank[i]);
            state[i] = 1;
        }
        CostSum cost(net.count_bits);
        for (int32_t k = 0; k < int32_t(merges.size()); ++k) {
            const int32_t a = merges[k].first, b = merges[k].second, c = n_init + k;
            if (a < 0 || b < 0 || a >= c || b >= c || a == b) return TN_EINVAL;
            if (state[a] != 1 || state[b] != 1) return TN_EINVAL;
            state[a] = state[b] = 2;
            state[c] = 1;
            const uint64_t *ba = bits.data() + size_t(a) * W, *bb = bits.data() + size_t(b) * W;
            uint64_t* bc = bits.data() + size_t(c) * W;
            int32_t rC = 0;
            for (int32_t w = 0; w < W; ++w) {
                bc[w] = ba[w] ^ bb[w];
                rC += __builtin_popcountll(bc[w]);
            }
            if (rC > TN_MAX_RANK) return TN_ERANK;
            rank[c] = rC;
            cost.add(rank[a], rank[b], (rank[a] + rank[b] - rC) / 2, rC);
            maxr = std::max(maxr, rC);
        }
        int32_t live = 0, root = -1;
        for (int32_t i = 0; i < n_ids; ++i)
            if (state[i] == 1) {
                ++live;
                root = i;
            }
        if (n_ids > 0 && live != 1) return TN_EINVAL;
        if (root >= 0 && rank[root] != 0) return TN_EINVAL;  // open bonds left
        plan = Plan{};
        plan.n_init = n_init;
        plan.n_vars = net.n_vars;
        plan.count_bits = net.count_bits;
        plan.max_entry = net.max_entry;
        plan.merges = std::move(merges);
        plan.root = root;
        plan.sketch = true;
        plan.cost_us = cost.t;
        plan.stats.n_steps = int32_t(plan.merges.size());
        plan.stats.max_rank = maxr;
        plan.stats.log2_cost = cost.t > 0 ? std::log2(cost.t) : 0.0;
        plan.stats.chosen = chosen;
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

tn_status make_plan(const Network& net, std::vector<std::pair<int32_t, int32_t>> merges, int32_t chosen,
                    Plan& plan) {
    try {
        const int32_t n_init = int32_t(net.t.size());
        plan = Plan{};
        plan.n_init = n_init;
        plan.n_vars = net.n_vars;
        plan.count_bits = net.count_bits;
        plan.max_entry = net.max_entry;
        const int32_t n_bonds = int32_t(net.bond_end.size());
        const int32_t n_ids = n_init + int32_t(merges.size());
        // --- validate the merge list and compute bond sets
        std::vector<std::vector<int32_t>> bset(n_ids);
        std::vector<int8_t> state(n_ids, 0);  // 0 unborn, 1 live, 2 consumed
        for (int32_t i = 0; i < n_init; ++i) {
            bset[i] = net.t[i].bonds;
            std::sort(bset[i].begin(), bset[i].end());
            if (std::adjacent_find(bset[i].begin(), bset[i].end()) != bset[i].end()) return TN_EINVAL;
            state[i] = 1;
        }
        std::vector<int32_t> death(n_bonds, -1);
        for (int32_t k = 0; k < int32_t(merges.size()); ++k) {
            int32_t a = merges[k].first, b = merges[k].second;
            if (a < 0 || b < 0 || a >= n_init + k || b >= n_init + k || a == b) return TN_EINVAL;
            if (state[a] != 1 || state[b] != 1) return TN_EINVAL;
            state[a] = state[b] = 2;
            state[n_init + k] = 1;
            std::vector<int32_t>& c = bset[n_init + k];
            std::set_symmetric_difference(bset[a].begin(), bset[a].end(), bset[b].begin(), bset[b].end(),
                                          std::back_inserter(c));
            std::vector<int32_t> sh;
            std::set_intersection(bset[a].begin(), bset[a].end(), bset[b].begin(), bset[b].end(),
                                  std::back_inserter(sh));
            for (int32_t x : sh) death[x] = k;
            if (int32_t(c.size()) > TN_MAX_RANK) return TN_ERANK;
        }
        int32_t live = 0, root = -1;
        for (int32_t i = 0; i < n_ids; ++i)
            if (state[i] == 1) {
                ++live;
                root = i;
            }
        if (n_ids > 0 && live != 1) return TN_EINVAL;
        if (root >= 0 && !bset[root].empty()) return TN_EINVAL;  // open bonds left
        plan.root = root;
        plan.merges = merges;
        // --- layouts: bonds by (death, id)
        plan.layout.resize(n_ids);
        plan.rank.resize(n_ids);
        for (int32_t i = 0; i < n_ids; ++i) {
            std::vector<int32_t> l = bset[i];
            std::sort(l.begin(), l.end(), [&](int32_t x, int32_t y) {
                return death[x] != death[y] ? death[x] < death[y] : x < y;
            });
            plan.rank[i] = int32_t(l.size());
            plan.layout[i] = std::move(l);
        }
        // --- init region
        plan.init_off.assign(n_init, 0);
        int64_t io = 0;
        for (int32_t i = 0; i < n_init; ++i) {
            plan.init_off[i] = io;
            io += align_up(int64_t(1) << plan.rank[i]);
        }
        plan.init_elems = io;
        // --- steps, levels and arena
        std::vector<int32_t> level(n_ids, 0);
        std::vector<int64_t> off(n_ids, -1);
        Arena arena;
        plan.steps.reserve(merges.size());
        double entries = 0, macs = 0;
        int32_t maxr = 0;
        for (int32_t i = 0; i < n_init; ++i) maxr = std::max(maxr, plan.rank[i]);
        for (int32_t k = 0; k < int32_t(merges.size()); ++k) {
            Step st;
            st.a = merges[k].first;
            st.b = merges[k].second;
            st.out = n_init + k;
            st.rA = plan.rank[st.a];
            st.rB = plan.rank[st.b];
            st.rC = plan.rank[st.out];
            st.s = (st.rA + st.rB - st.rC) / 2;
            const auto& LA = plan.layout[st.a];
            const auto& LB = plan.layout[st.b];
            for (int32_t z = 0; z < st.s; ++z)
                if (LA[z] != LB[z]) return TN_EINVAL;  // cannot happen by construction
            // C = merge of A[s..] and B[s..] in (death, id) order
            size_t ia = size_t(st.s), ib = size_t(st.s);
            int32_t j = 0;
            const auto& LC = plan.layout[st.out];
            uint64_t mask = 0;
            for (; j < st.rC; ++j) {
                int32_t bnd = LC[j];
                if (ia < LA.size() && LA[ia] == bnd) {
                    mask |= uint64_t(1) << j;
                    ++ia;
                } else if (ib < LB.size() && LB[ib] == bnd) {
                    ++ib;
                } else {
                    return TN_EINVAL;
                }
            }
            st.maskA = mask;
            st.initA = st.a < n_init;
            st.initB = st.b < n_init;
            st.level = 1 + std::max(level[st.a], level[st.b]);
            level[st.out] = st.level;
            int64_t szC = align_up(int64_t(1) << st.rC);
            st.offC = arena.alloc(szC);
            off[st.out] = st.offC;
            st.offA = st.initA ? plan.init_off[st.a] : off[st.a];
            st.offB = st.initB ? plan.init_off[st.b] : off[st.b];
            if (!st.initA) arena.release(off[st.a], align_up(int64_t(1) << st.rA));
            if (!st.initB) arena.release(off[st.b], align_up(int64_t(1) << st.rB));
            entries += std::ldexp(1.0, st.rA) + std::ldexp(1.0, st.rB) + std::ldexp(1.0, st.rC);
            macs += std::ldexp(1.0, st.rA + st.rB - st.s);
            maxr = std::max(maxr, st.rC);
            plan.steps.push_back(st);
        }
        plan.arena_elems = arena.high;
        // wave layout: steps of one level run concurrently, so every output
        // of a wave is allocated before any input consumed in it is released
        {
            int32_t maxl = 0;
            for (const Step& st : plan.steps) maxl = std::max(maxl, st.level);
            std::vector<std::vector<int32_t>> by_level(size_t(maxl) + 1);
            for (int32_t k = 0; k < int32_t(plan.steps.size()); ++k) by_level[plan.steps[k].level].push_back(k);
            std::vector<int64_t> woff(n_ids, -1);
            Arena wa;
            for (int32_t L = 1; L <= maxl; ++L) {
                for (int32_t k : by_level[L]) {
                    Step& st = plan.steps[k];
                    st.woffC = wa.alloc(align_up(int64_t(1) << st.rC));
                    woff[st.out] = st.woffC;
                }
                for (int32_t k : by_level[L]) {
                    Step& st = plan.steps[k];
                    st.woffA = st.initA ? plan.init_off[st.a] : woff[st.a];
                    st.woffB = st.initB ? plan.init_off[st.b] : woff[st.b];
                }
                for (int32_t k : by_level[L]) {
                    const Step& st = plan.steps[k];
                    if (!st.initA) wa.release(woff[st.a], align_up(int64_t(1) << st.rA));
                    if (!st.initB) wa.release(woff[st.b], align_up(int64_t(1) << st.rB));
                }
            }
            plan.warena_elems = wa.high;
        }
        plan.stats.n_steps = int32_t(plan.steps.size());
        plan.stats.max_rank = maxr;
        plan.stats.entries = entries;
        plan.stats.macs = macs;
        plan.stats.peak_elems = uint64_t(plan.arena_elems + plan.init_elems);
        const double c = plan_cost(plan);
        plan.cost_us = c;
        plan.stats.log2_cost = c > 0 ? std::log2(c) : 0.0;
        plan.stats.chosen = chosen;
        plan.stats.fallback = 0;
    } catch (const std::bad_alloc&) {
        return TN_ENOMEM;
    }
    return TN_OK;
}

}  // namespace tn

namespace tn {

// Checks both arena layouts against the liveness of the plan's tensors: no
// tensor may overlap another one that is alive at the same time, in plan
// order (one step at a time) and in waves (all steps of a level at once).
tn_status verify_plan(const Plan& plan) {
    const int32_t n_init = plan.n_init;
    const int32_t n_ids = n_init + int32_t(plan.steps.size());
    std::vector<int32_t> born(n_ids, -1), died(n_ids, -1), lborn(n_ids, 0), ldied(n_ids, 0);
    std::vector<int64_t> off(n_ids, -1), woff(n_ids, -1), size(n_ids, 0);
    for (int32_t k = 0; k < int32_t(plan.steps.size()); ++k) {
        const Step& st = plan.steps[k];
        born[st.out] = k;
        lborn[st.out] = st.level;
        died[st.a] = died[st.b] = k;
        ldied[st.a] = ldied[st.b] = st.level;
        off[st.out] = st.offC;
        woff[st.out] = st.woffC;
        size[st.out] = int64_t(1) << st.rC;
        if (st.offC < 0 || st.offC + size[st.out] > plan.arena_elems) return TN_EINVAL;
        if (st.woffC < 0 || st.woffC + size[st.out] > plan.warena_elems) return TN_EINVAL;
        if (!st.initA && (st.offA != off[st.a] || st.woffA != woff[st.a])) return TN_EINVAL;
        if (!st.initB && (st.offB != off[st.b] || st.woffB != woff[st.b])) return TN_EINVAL;
    }
    const int32_t root = plan.root;
    if (root >= n_init) {
        died[root] = int32_t(plan.steps.size());
        ldied[root] = 1 << 30;
    }
    for (int32_t x = n_init; x < n_ids; ++x)
        for (int32_t y = x + 1; y < n_ids; ++y) {
            // plan order: live on [born, died] (inputs stay live through the step)
            const bool seq_overlap = born[x] <= died[y] && born[y] <= died[x];
            const bool wave_overlap = lborn[x] <= ldied[y] && lborn[y] <= ldied[x];
            const bool mem = off[x] < off[y] + size[y] && off[y] < off[x] + size[x];
            const bool wmem = woff[x] < woff[y] + size[y] && woff[y] < woff[x] + size[x];
            if ((seq_overlap && mem) || (wave_overlap && wmem)) return TN_EINVAL;
        }
    return TN_OK;
}

}  // namespace tn
